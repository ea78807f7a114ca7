// Batch planning (host only, no GPU calls): compiled network programs ->
// the arrays the kernels read, the executor of every network, the level
// executor's items and task queue, and the device workspace layout.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <array>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>

#include "batch.hpp"

namespace qtn {

NetLayout make_layout(const Net &net) {
  NetLayout lay;
  lay.coff.resize(net.consts.size());
  lay.poff.resize(net.ptensors.size());
  int64_t pos = 0;
  for (size_t c = 0; c < net.consts.size(); ++c) {
    lay.coff[c] = pos;
    pos += (int64_t)net.consts[c].size();
  }
  lay.n_const = pos;
  for (size_t t = 0; t < net.ptensors.size(); ++t) {
    lay.poff[t] = pos;
    pos += (int64_t)1 << net.ptensors[t].bits;
  }
  lay.leaf_region = pos;
  lay.ptens_elems = pos - lay.n_const;
  const Plan &p = net.gplan;
  lay.arena[0] = layout_buffers(p, p.n_fwd_ops, lay.off[0]);
  lay.arena[1] = layout_buffers(p, (int)p.ops.size(), lay.off[1]);
  return lay;
}

static int64_t abs_off(const Net &net, const NetLayout &lay, int variant, int v) {
  if (v < net.gplan.n_leaves) {
    int src = net.leaves[v].src;
    return src >= 0 ? lay.coff[src] : lay.poff[-src - 1];
  }
  return lay.leaf_region + lay.off[variant][v];
}

static int slot_for(HostProgram &hp, const ParamTensor &pt) {
  auto key = std::make_tuple(pt.kind, pt.param, pt.coeff, pt.folded + 2 * pt.diag);
  auto it = hp.slot_of.find(key);
  if (it != hp.slot_of.end()) return it->second;
  DParam s{};
  s.kind = pt.kind;
  s.param = pt.param;
  s.folded = pt.folded;
  s.diag = pt.diag;
  s.bits = pt.bits;
  s.off = hp.per_set;
  s.coeff = pt.coeff;
  hp.slots.push_back(s);
  hp.slot_of.emplace(key, hp.per_set);
  int r = hp.per_set;
  hp.per_set += 1 << pt.bits;
  return r;
}

static int append_consts(const Net &net, HostProgram &hp) {
  const int begin = (int)(hp.consts.size() / 2);
  for (auto &c : net.consts)
    for (auto &z : c) {
      hp.consts.push_back(z.real());
      hp.consts.push_back(z.imag());
    }
  return begin;
}

// Emit the ops of one variant with offsets from `boff`; LEAFGRAD targets
// are resolved by `leafgrad`.
template <typename BOff, typename LG>
static void emit_ops(const Plan &p, int n_ops, HostProgram &hp, BOff boff, LG leafgrad) {
  for (int i = 0; i < n_ops; ++i) {
    const Op &op = p.ops[i];
    DOp d{};
    d.type = op.type;
    d.nFX = op.nFX;
    d.nS = op.nS;
    d.nFY = op.nFY;
    d.maskX = op.maskX_F;
    d.maskY = op.maskY_F;
    d.nB = op.nB;
    d.tab = (int32_t)hp.tabs.size();
    hp.tabs.insert(hp.tabs.end(), op.tab.begin(), op.tab.end());
    d.tabB = (int32_t)hp.tabs.size();
    hp.tabs.insert(hp.tabs.end(), op.tabB.begin(), op.tabB.end());
    if (op.type == OP_CONTRACT) {
      d.x = boff(op.x);
      d.y = boff(op.y);
      d.z = boff(op.z);
    } else if (op.type == OP_SCALAR) {
      d.x = boff(op.x);
      d.y = boff(op.y);
      d.z = op.z;
    } else if (op.type == OP_SEED) {
      d.z = boff(op.z);
      d.aux0 = op.aux0;
    } else {
      d.x = boff(op.x);
      leafgrad(op, d);
    }
    hp.ops.push_back(d);
  }
}

// LDS bytes the fused adjoint program of a network needs.
static int64_t fused_lds_need(const Net &net, const NetLayout &lay, int eb, int n_params) {
  int64_t mem = lay.leaf_region + std::max(lay.arena[0], lay.arena[1]);
  return mem * eb + 256 * eb + (int64_t)std::max(1, net.gplan.n_components) * 16 + (int64_t)n_params * 8 + 256 + 64;
}

static uint32_t host_pdep(uint32_t v, uint32_t mask) {
  uint32_t out = 0;
  while (mask) {
    uint32_t low = mask & (0u - mask);
    if (v & 1u) out |= low;
    v >>= 1;
    mask ^= low;
  }
  return out;
}

// Operand offsets (X, Y) of output c of a contraction: c = (i, b, j) with i
// the X-only bits, b the batch bits (offset table), j the Y-only bits.
static void out_offsets(const std::vector<int32_t> &tabs, const DOp &op, uint32_t c, int32_t &ox, int32_t &oy) {
  const uint32_t rest = c >> op.nFY;
  ox = op.x + (int32_t)host_pdep(rest >> op.nB, op.maskX);
  oy = op.y + (int32_t)host_pdep(c & ((1u << op.nFY) - 1u), op.maskY);
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    ox += tabs[op.tabB + 2 * b];
    oy += tabs[op.tabB + 2 * b + 1];
  }
}

// Lane record (see kRecLanes) of one op whose operands all sit in one
// memory at the op's offsets (below 2^16): 64 int4 appended to `recs`;
// returns its type (0: the op has no record form). `pt` are the network's
// parametric tensors (for leaf-gradient ops).
static int build_record(const std::vector<int32_t> &tabs, const std::vector<DParam> &pt, const DOp &op,
                        std::vector<int32_t> &recs) {
  auto pack = [](int32_t a, int32_t b) { return (a & 0xffff) | (b << 16); };
  {
    const int lgOut = op.nFX + op.nB + op.nFY;
    // LDS offsets of output c's X and Y rows
    auto offs = [&](uint32_t c, int32_t &ox, int32_t &oy) { out_offsets(tabs, op, c, ox, oy); };
    // (X, Y) offsets of summed entry k (tables of at most 2^12 entries)
    auto tab = [&](int k, int32_t &tx, int32_t &ty) {
      tx = tabs[op.tab + 2 * k];
      ty = tabs[op.tab + 2 * k + 1];
    };
    int type = 0, A = 0, B = 0, C = 0, zf = 0;
    int lgG = 0;
    if (op.type == OP_CONTRACT) {
      zf = op.z;
      if (lgOut <= 6 && op.nS <= 2) {
        type = kRecLite;
        A = op.nS;
        B = lgOut;
      } else if (op.nS == 0 && lgOut <= 8) {
        type = kRecWide;
        B = lgOut;
      } else if (lgOut <= 6 && op.nS <= 12) {
        lgG = std::min(6 - lgOut, op.nS);
        const int lgR = op.nS - lgG;
        bool additive = lgR <= 6;
        // entry k = g + G i must sit at t(g) + t(G i)
        for (int k = 0; additive && k < (1 << op.nS); ++k) {
          int32_t ax, ay, bx, by, cx, cy;
          tab(k, ax, ay);
          tab(k & ((1 << lgG) - 1), bx, by);
          tab(k & ~((1 << lgG) - 1), cx, cy);
          additive = ax == bx + cx && ay == by + cy;
        }
        if (additive) {
          type = kRecNarrow;
          A = lgG;
          B = lgOut;
          C = lgR;
        }
      }
    } else if (op.type == OP_SCALAR && op.nS <= 6) {
      type = kRecScalar;
      A = op.nS;
      zf = op.z;
    } else if (op.type == OP_SEED) {
      type = kRecSeed;
      zf = op.z;
    } else if (op.type == OP_LEAFGRAD && op.nFX <= 8) {
      type = kRecLeafGrad;
      B = op.nFX;
      zf = pt[op.aux0].param;
    }
    if (zf >= (1 << 17)) type = 0;
    for (int l = 0; l < kRecLanes; ++l) {
      int32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      if (type == kRecLite) {
        if (l < (1 << lgOut)) offs((uint32_t)l, a0, a1);
        if (l < (1 << op.nS)) {
          int32_t tx, ty;
          tab(l, tx, ty);
          a2 = pack(tx, ty);
        }
      } else if (type == kRecWide) {
        offs((uint32_t)l, a0, a1);
        if (l >= 1 && (l << 6) < (1 << lgOut)) {  // offset steps of outputs 64 l
          int32_t dx, dy;
          offs((uint32_t)(l << 6), dx, dy);
          a3 = pack(dx - op.x, dy - op.y);
        }
      } else if (type == kRecNarrow) {
        // lane l sums entries g + G i (g = l mod G) of output l / G
        const int j = l >> lgG, g = l & ((1 << lgG) - 1);
        if (j < (1 << lgOut)) {
          int32_t tx, ty;
          offs((uint32_t)j, a0, a1);
          tab(g, tx, ty);
          a0 += tx;
          a1 += ty;
        } else {
          a0 = op.x;
          a1 = op.y;
        }
        if (l < (1 << C)) {
          int32_t tx, ty;
          tab(l << lgG, tx, ty);
          a2 = pack(tx, ty);
        }
      } else if (type == kRecScalar) {
        int32_t tx = 0, ty = 0;
        if (l < (1 << op.nS)) tab(l, tx, ty);
        a0 = op.x + tx;
        a1 = op.y + ty;
      } else if (type == kRecSeed) {
        if (l == 0) a0 = op.aux0;
      } else if (type == kRecLeafGrad) {
        a0 = op.x + l;
        for (int q = 0; q < 4; ++q)
          if (l + (q << 6) < (1 << op.nFX)) a1 |= (tabs[op.tab + l + (q << 6)] & 0xff) << (8 * q);
        const DParam &d = pt[op.aux0];
        int64_t bits;
        std::memcpy(&bits, &d.coeff, sizeof(bits));
        if (l == 0) a2 = d.slot;
        if (l == 1) a2 = (int32_t)(bits & 0xffffffff);
        if (l == 2) a2 = (int32_t)(bits >> 32);
      }
      if (l == 0) a3 = type ? (type | (A << 3) | (B << 7) | (C << 11) | (zf << 15)) : 0;
      recs.push_back(a0);
      recs.push_back(a1);
      recs.push_back(a2);
      recs.push_back(a3);
    }
    return type;
  }
}

// Lane records of ops [first, first + n) of `loc` (LDS offsets).
static void build_records(const HostProgram &loc, const std::vector<DParam> &pt, int first, int n,
                          std::vector<int32_t> &recs) {
  for (int o = first; o < first + n; ++o) build_record(loc.tabs, pt, loc.ops[o], recs);
}

// Set-packed records (see kSetContract), 2^lgW lanes per set, of the ops of
// `loc`; false when some op has no set-packed form (its record is then
// left empty).
static bool build_set_records(const HostProgram &loc, const std::vector<DParam> &pt, int lgW,
                              std::vector<int32_t> &recs) {
  const int W = 1 << lgW, lgGmax = std::min(lgW, kLgMaxGroupLanes);
  auto pack = [](int32_t a, int32_t b) { return (a & 0xffff) | (b << 16); };
  bool all = true;
  for (const DOp &op : loc.ops) {
    std::vector<std::array<int32_t, 4>> f(W, std::array<int32_t, 4>{0, 0, 0, 0});
    auto offs = [&](uint32_t c, int32_t &ox, int32_t &oy) { out_offsets(loc.tabs, op, c, ox, oy); };
    auto tab = [&](int k, int32_t &tx, int32_t &ty) {
      tx = loc.tabs[op.tab + 2 * k];
      ty = loc.tabs[op.tab + 2 * k + 1];
    };
    // entry k = g + G i must sit at t(g) + t(G i)
    auto additive = [&](int nS, int lgG) {
      const int lo = (1 << lgG) - 1;
      for (int k = 0; k < (1 << nS); ++k) {
        int32_t ax, ay, bx, by, cx, cy;
        tab(k, ax, ay);
        tab(k & lo, bx, by);
        tab(k & ~lo, cx, cy);
        if (ax != bx + cx || ay != by + cy) return false;
      }
      return true;
    };
    int type = 0, lgG = 0, lgQ = 0, lgR = 0, lgOut = 0, zf = 0;
    if (op.type == OP_CONTRACT && op.nS <= 12) {
      lgOut = op.nFX + op.nB + op.nFY;
      lgG = lgOut >= lgW ? 0 : std::min(std::min(lgW - lgOut, op.nS), lgGmax);
      lgQ = std::max(0, lgOut - lgW);
      lgR = op.nS - lgG;
      // outputs w / G + (W / G) q must cover all outputs once
      if (lgQ > 0 && lgG > 0) lgQ = 99;
      if (lgOut < lgW && lgOut + lgG > lgW) lgQ = 99;
      if (lgQ <= std::min(lgW, 7) && lgR <= std::min(lgW, 7) && additive(op.nS, lgG)) {
        type = kSetContract;
        zf = op.z;
        for (int w = 0; w < W; ++w) {
          const int j = w >> lgG, g = w & ((1 << lgG) - 1);
          int32_t tx, ty;
          if (j < (1 << lgOut)) {
            offs((uint32_t)j, f[w][0], f[w][1]);
            tab(g, tx, ty);
            f[w][0] += tx;
            f[w][1] += ty;
          } else {
            f[w][0] = op.x;
            f[w][1] = op.y;
          }
          if (w < (1 << lgR)) {
            tab(w << lgG, tx, ty);
            f[w][2] = pack(tx, ty);
          }
          if (w >= 1 && w < (1 << lgQ)) {
            offs((uint32_t)(w * W), tx, ty);
            f[w][3] = pack(tx - op.x, ty - op.y);
          }
        }
      }
    } else if (op.type == OP_SCALAR && op.nS <= 12) {
      lgG = std::min(lgGmax, op.nS);
      lgR = op.nS - lgG;
      if (lgR <= std::min(lgW, 7) && additive(op.nS, lgG)) {
        type = kSetScalar;
        zf = op.z;
        for (int w = 0; w < W; ++w) {
          int32_t tx = 0, ty = 0;
          if (w < (1 << lgG)) tab(w, tx, ty);
          f[w][0] = op.x + tx;
          f[w][1] = op.y + ty;
          if (w < (1 << lgR)) {
            tab(w << lgG, tx, ty);
            f[w][2] = pack(tx, ty);
          }
        }
      }
    } else if (op.type == OP_SEED) {
      type = kSetSeed;
      zf = op.z;
      f[0][0] = op.aux0;
    } else if (op.type == OP_LEAFGRAD && op.nFX <= 8) {
      lgG = std::min(lgGmax, op.nFX);
      lgR = op.nFX - lgG;
      auto perm = [&](int e) { return loc.tabs[op.tab + e]; };
      bool add = lgR <= std::min(lgW, 7);
      for (int e = 0; add && e < (1 << op.nFX); ++e)
        add = perm(e) == perm(e & ((1 << lgG) - 1)) + perm(e & ~((1 << lgG) - 1));
      if (add) {
        type = kSetLeafGrad;
        const DParam &d = pt[op.aux0];
        zf = d.param;
        int64_t bits;
        std::memcpy(&bits, &d.coeff, sizeof(bits));
        for (int w = 0; w < W; ++w) {
          const bool act = w < (1 << lgG);
          f[w][0] = op.x + (act ? w : 0);
          f[w][1] = act ? perm(w) : 0;
          if (w < (1 << lgR)) f[w][2] = perm(w << lgG);
        }
        f[1][3] = d.slot;
        f[2][3] = (int32_t)(bits & 0xffffffff);
        f[3][3] = (int32_t)(bits >> 32);
      }
    }
    if (zf >= (1 << 16)) type = 0;
    if (type == 0) all = false;
    f[0][3] = type ? (int32_t)((uint32_t)type | (lgG << 3) | (lgQ << 6) | (lgR << 9) | (lgOut << 12) |
                               ((uint32_t)zf << 16))
                   : 0;
    for (int w = 0; w < W; ++w)
      for (int c = 0; c < 4; ++c) recs.push_back(f[w][c]);
  }
  return all;
}

// Append the fused programs (forward, forward+adjoint) of one network.
// Networks whose programs are identical (same ops, offset tables, constants
// and parametric tensors: e.g. isomorphic light cones contracted in the same
// order) share one copy, which keeps the descriptors of a batch small enough
// to stay in the scalar cache.
static void append_fused(const Net &net, const NetLayout &lay, HostProgram &hp, bool gmem) {
  const Plan &p = net.gplan;
  HostProgram loc;  // this network's program with local indices
  std::vector<DParam> lptens;
  for (size_t t = 0; t < net.ptensors.size(); ++t) {
    const ParamTensor &pt = net.ptensors[t];
    DParam d{};
    d.kind = pt.kind;
    d.param = pt.param;
    d.folded = pt.folded;
    d.diag = pt.diag;
    d.bits = pt.bits;
    d.off = (int32_t)lay.poff[t];
    d.goff = (int32_t)(lay.poff[t] - lay.n_const);
    d.coeff = pt.coeff;
    d.slot = slot_for(hp, pt);
    lptens.push_back(d);
  }
  int op_begin[2], n_ops[2];
  for (int variant = 0; variant < 2; ++variant) {
    op_begin[variant] = (int)loc.ops.size();
    n_ops[variant] = variant == 0 ? p.n_fwd_ops : (int)p.ops.size();
    emit_ops(
        p, n_ops[variant], loc, [&](int v) { return (int32_t)abs_off(net, lay, variant, v); },
        [&](const Op &op, DOp &d) { d.aux0 = op.aux0; });
  }
  append_consts(net, loc);
  std::string sig;
  auto put = [&](const void *q, size_t n) { sig.append(reinterpret_cast<const char *>(q), n); };
  put(loc.ops.data(), loc.ops.size() * sizeof(DOp));
  put(loc.tabs.data(), loc.tabs.size() * sizeof(int32_t));
  put(loc.consts.data(), loc.consts.size() * sizeof(double));
  put(lptens.data(), lptens.size() * sizeof(DParam));
  put(n_ops, sizeof(n_ops));
  auto it = hp.program_of.find(sig);
  if (it != hp.program_of.end()) {
    hp.nets_fwd.push_back(hp.nets_fwd[it->second]);
    hp.nets_grad.push_back(hp.nets_grad[it->second]);
    return;
  }
  const int tab0 = (int)hp.tabs.size(), op0 = (int)hp.ops.size(), ptens_begin = (int)hp.ptens.size();
  const int rec0 = (int)(hp.recs.size() / (4 * kRecLanes));
  build_records(loc, lptens, 0, (int)loc.ops.size(), hp.recs);
  for (int variant = 0; variant < 2; ++variant)
    for (int o = op_begin[variant]; o < op_begin[variant] + n_ops[variant]; ++o)
      if (hp.recs[((size_t)(rec0 + o) * kRecLanes) * 4 + 3] == 0 && !gmem) hp.generic[variant] = true;
  for (int i = 0; i < 2; ++i)
    if (!build_set_records(loc, lptens, i == 0 ? 4 : 5, hp.srecs[i]) && !gmem) hp.sets_ok[i] = false;
  const int const_begin = (int)(hp.consts.size() / 2);
  for (DOp d : loc.ops) {
    d.tab += tab0;
    d.tabB += tab0;
    if (d.type == OP_LEAFGRAD) d.aux0 += ptens_begin;
    hp.ops.push_back(d);
  }
  hp.tabs.insert(hp.tabs.end(), loc.tabs.begin(), loc.tabs.end());
  hp.consts.insert(hp.consts.end(), loc.consts.begin(), loc.consts.end());
  hp.ptens.insert(hp.ptens.end(), lptens.begin(), lptens.end());
  hp.max_ptens_elems = std::max(hp.max_ptens_elems, (int)lay.ptens_elems);
  for (int variant = 0; variant < 2; ++variant) {
    DNet dn{};
    dn.op_begin = op0 + op_begin[variant];
    dn.rec_begin = rec0 + op_begin[variant];
    dn.n_ops = n_ops[variant];
    dn.n_comp = p.n_components;
    dn.mem_elems = (int32_t)(lay.leaf_region + lay.arena[variant]);
    dn.const_begin = const_begin;
    dn.n_const = (int32_t)lay.n_const;
    dn.ptens_begin = ptens_begin;
    dn.n_ptens = (int32_t)net.ptensors.size();
    (variant == 0 ? hp.nets_fwd : hp.nets_grad).push_back(dn);
    if (gmem) {
      hp.max_mem_g[variant] = std::max<int64_t>(hp.max_mem_g[variant], dn.mem_elems);
    } else {
      int &mx = variant == 0 ? hp.max_mem_fwd : hp.max_mem_grad;
      mx = std::max(mx, dn.mem_elems);
    }
  }
  hp.program_of.emplace(sig, (int)hp.nets_fwd.size() - 1);
  hp.n_programs++;
  hp.max_comp = std::max(hp.max_comp, p.n_components);
}

// A network on the level executor: buffers in a global arena slice per
// parameter vector; adjoint accumulators after the arena.
static LevelNet append_level(const Net &net, const NetLayout &lay, HostProgram &hp, int index, int eb,
                             int64_t budget_bytes, int max_sets) {
  const Plan &p = net.gplan;
  LevelNet ln;
  ln.net = index;
  ln.n_comp = p.n_components;
  ln.const_begin = append_consts(net, hp);
  ln.n_const = (int)lay.n_const;
  ln.stride[0] = lay.leaf_region + lay.arena[0];
  ln.gbar_begin = lay.leaf_region + lay.arena[1];
  ln.ptens_elems = lay.ptens_elems;
  ln.leaf_region = lay.leaf_region;
  ln.stride[1] = ln.gbar_begin + lay.ptens_elems;
  for (int v = 0; v < 2; ++v) ln.stride[v] = (ln.stride[v] + 63) & ~int64_t(63);
  ln.ptens_begin = (int)hp.ptens.size();
  ln.n_ptens = (int)net.ptensors.size();
  for (size_t t = 0; t < net.ptensors.size(); ++t) {
    const ParamTensor &pt = net.ptensors[t];
    DParam d{};
    d.kind = pt.kind;
    d.param = pt.param;
    d.folded = pt.folded;
    d.diag = pt.diag;
    d.bits = pt.bits;
    d.off = (int32_t)lay.poff[t];
    d.goff = ln.gbar_begin + lay.poff[t] - lay.n_const;
    d.coeff = pt.coeff;
    d.slot = slot_for(hp, pt);
    hp.ptens.push_back(d);
  }
  for (int variant = 0; variant < 2; ++variant) {
    ln.op_begin[variant] = (int)hp.ops.size();
    ln.n_ops[variant] = variant == 0 ? p.n_fwd_ops : (int)p.ops.size();
    emit_ops(
        p, ln.n_ops[variant], hp, [&](int v) { return abs_off(net, lay, variant, v); },
        [&](const Op &op, DOp &d) {
          d.y = ln.gbar_begin + lay.poff[op.aux0] - lay.n_const;
          d.aux0 = ln.ptens_begin + op.aux0;
          d.aux1 = op.aux1;
        });
  }
  // a set's region past kMaxLevelElems elements leaves the network usable
  // for forward passes only
  ln.grad_ok = ln.stride[1] < kMaxLevelElems;
  int64_t per = ln.stride[ln.grad_ok ? 1 : 0] * eb;
  ln.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(max_sets, budget_bytes / std::max<int64_t>(1, per)));
  ln.cost = p.flops + p.flops_grad;
  return ln;
}

// --- matrix-core eligibility and tile shapes --------------------------------------------------

// True when the matrix-core path takes this op: no batch bits, at least 16
// summed entries; complex64: both free indices at least 4 wide and one at
// least 64 wide (tiles 64 x 64, 16 x 64 or 64 x 16; a 4- or 8-wide index is
// one padded 16-wide tile), or both narrower than 64 with at least 64
// summed entries (one 16 x 64 tile whose columns past the Y index read
// aliased entries and are not written: a long sum on few outputs is
// latency-bound on the vector units); complex128: both at least 64 wide
// (64 x 64 tiles).
bool mfma_eligible(int dtype, const DOp &op) {
  if (op.type != OP_CONTRACT || op.nB != 0 || op.nS < 4) return false;
  if (dtype == TN_C128) return op.nFX >= 6 && op.nFY >= 6;
  return dtype == TN_C64 && op.nFX >= 2 && op.nFY >= 2 && (op.nFX >= 6 || op.nFY >= 6 || op.nS >= 6);
}

// Tile of an eligible op: shape 0 by its free-index widths (above), else
// the tuner's choice, 1 = 64 x 64, 2 = 16 x 64, 3 = 64 x 16 (any of them
// covers any eligible op: a side wider than its index reads aliased
// entries and does not write them).
static inline int tile_m(const DOp &op, int shape) { return shape ? (shape == 2 ? 16 : 64) : op.nFX >= 6 ? 64 : 16; }
static inline int tile_n(const DOp &op, int shape) {
  return shape ? (shape == 3 ? 16 : 64) : op.nFY >= 6 || op.nFX < 6 ? 64 : 16;
}

// Output tiles of an eligible op per parameter vector.
int mfma_tiles(const DOp &op, int shape) {
  const int lm = tile_m(op, shape) == 64 ? 6 : 4, ln = tile_n(op, shape) == 64 ? 6 : 4;
  return 1 << ((op.nFX > lm ? op.nFX - lm : 0) + (op.nFY > ln ? op.nFY - ln : 0));
}

// Kernel variant of an op: bit 0 XK (X's lowest address bit is summed), bit 1
// YK, bit 2 BM = 16, bit 3 BN = 16, bit 4 split-BF16, bit 5 FP64.
int mfma_variant(const DOp &op, int prec, int shape) {
  return (!(op.maskX & 1u) ? 1 : 0) | (!(op.maskY & 1u) ? 2 : 0) | (tile_m(op, shape) == 16 ? 4 : 0) |
         (tile_n(op, shape) == 16 ? 8 : 0) | (prec == TN_MFMA_BF16X3 ? 16 : 0) | (prec == TN_MFMA_FP64 ? 32 : 0);
}

// Key of a large op for the autotuner: dtype, precision, free/summed bit
// counts and which operands are read with the summed index contiguous.
std::string shape_class(int dtype, const DOp &op, int prec) {
  return std::to_string(dtype) + "p" + std::to_string(prec) + ":" + std::to_string(op.nFX) + "," + std::to_string(op.nS) +
         "," + std::to_string(op.nFY) + ":" + std::to_string(!(op.maskX & 1u)) + std::to_string(!(op.maskY & 1u));
}

// Matrix-core precision a level op runs with (0: the thin path).
int level_prec(const ItemCtx &c, const DOp &op) {
  if (!mfma_eligible(c.dtype, op)) return 0;
  if (c.all_thin) return 0;
  if (!c.use_mfma) return c.mfma_prec;
  auto it = c.use_mfma->find(shape_class(c.dtype, op, c.mfma_prec));
  return it == c.use_mfma->end() || it->second ? c.mfma_prec : 0;
}

int level_prec(const tn_batch *b, const DOp &op) { return level_prec(item_ctx(b), op); }

// Tile shape of a matrix-core level op: the tuner's choice (its class's
// value 2-4 is shape 1-3), else by the op's widths (0). complex128 has 64 x
// 64 tiles only.
int level_tile(const ItemCtx &c, const DOp &op) {
  if (c.dtype == TN_C128) return 0;
  if (c.force_tile >= 0) return c.force_tile;
  if (!c.use_mfma) return 0;
  auto it = c.use_mfma->find(shape_class(c.dtype, op, c.mfma_prec));
  return it != c.use_mfma->end() && it->second >= 2 && it->second <= 4 ? it->second - 1 : 0;
}

ItemCtx item_ctx(const tn_batch *b) {
  ItemCtx c;
  c.dtype = b->dtype;
  c.mfma_prec = b->mfma_prec;
  c.split_target = b->split_target;
  c.use_mfma = &b->use_mfma;
  c.ops = &b->hp.ops;
  c.tabs = &b->hp.tabs;
  return c;
}

// --- LDS residency of the task executor -------------------------------------------------------

// Which tensors of one network program (variant v) a task-executor
// workgroup keeps in its LDS arena of c.lds_elems elements, per op: a0 flags
// (kLdsX / kLdsY / kLdsZ) and the LDS element offsets of those operands.
// The leaf region is mirrored to LDS [0, leaf region) when it takes at most
// half the arena. An intermediate is a candidate when every op that writes
// or reads it runs on the vector units (a thin contraction, or a leaf
// adjoint reading it); the matrix-core tiles, rank-0 sums and seeds read and
// write global memory. Candidates take arena space first-fit when written
// and give it back after their last read; one that does not fit goes to the
// tile staging after the arena (c.tile_elems elements) when no matrix-core
// product runs while it lives, else stays in the region. Tensors are told apart by their region offset (a write at an
// offset starts a new tensor there). With gradients (v = 1) the adjoint
// accumulators of the parametric tensors take a fixed block after the
// mirror, for the whole program (*acc_at: its LDS offset, else -1), so
// leaf adjoints add into LDS.
struct LdsOp {
  int32_t flags = 0, x = 0, y = 0, z = 0;
};

static bool lds_mirror(const ItemCtx &c, const LevelNet &ln) {
  return c.one_wg && c.lds_elems > 0 && ln.leaf_region > 0 && 2 * ln.leaf_region <= c.lds_elems;
}

static std::vector<LdsOp> lds_assign(const ItemCtx &c, const LevelNet &ln, int v, int64_t *acc_at) {
  const int n = ln.n_ops[v];
  std::vector<LdsOp> res(n);
  *acc_at = -1;
  if (!c.one_wg || c.lds_elems <= 0) return res;
  const bool mirror = lds_mirror(c, ln);
  const int64_t leaf = ln.leaf_region;
  struct Inst {
    int64_t off, size;
    int last = -1;
    bool banned = false;
    int64_t lds = -1;
  };
  std::vector<Inst> inst;
  std::map<int64_t, int> cur;  // region offset -> current tensor there
  std::vector<std::array<int, 3>> uses(n, {-1, -1, -1});  // tensors read as X, Y and written as Z
  auto bits = [](int b) { return (int64_t)1 << b; };
  for (int k = 0; k < n; ++k) {
    const DOp &op = (*c.ops)[ln.op_begin[v] + k];
    const bool thin = op.type == OP_CONTRACT && level_prec(c, op) == 0;
    const bool vector_read = thin || op.type == OP_LEAFGRAD;
    auto read = [&](int64_t off, int slot) {
      if (off < leaf) return;
      auto it = cur.find(off);
      if (it == cur.end()) return;
      Inst &t = inst[it->second];
      t.last = k;
      if (!vector_read) t.banned = true;
      uses[k][slot] = it->second;
    };
    if (op.type == OP_CONTRACT || op.type == OP_SCALAR) {
      read(op.x, 0);
      read(op.y, 1);
    } else if (op.type == OP_LEAFGRAD) {
      read(op.x, 0);
    }
    if (op.type == OP_CONTRACT || op.type == OP_SEED) {
      Inst t;
      t.off = op.z;
      t.size = op.type == OP_SEED ? 1 : bits(op.nFX + op.nB + op.nFY);
      t.banned = !thin;
      cur[op.z] = (int)inst.size();
      uses[k][2] = (int)inst.size();
      inst.push_back(t);
    }
  }
  int64_t base = mirror ? ((leaf + 31) & ~int64_t(31)) : 0;
  if (v == 1 && ln.ptens_elems > 0 && 2 * (base + ln.ptens_elems) <= c.lds_elems) {
    *acc_at = base;
    base = (base + ln.ptens_elems + 31) & ~int64_t(31);
  }
  const int64_t cap = c.lds_elems - base;
  // the tile staging after the arena, past the reserve that rank-0 sums and
  // outputs use: for tensors whose whole life has no matrix-core product
  const int64_t tbase = c.lds_elems + kTileReserve / (c.dtype == TN_C128 ? 16 : 8), tcap = c.tile_elems;
  std::vector<int> tile_use(n + 1, 0);  // prefix counts of the matrix-core products
  for (int k = 0; k < n; ++k) {
    const DOp &op = (*c.ops)[ln.op_begin[v] + k];
    tile_use[k + 1] = tile_use[k] + (op.type == OP_CONTRACT && level_prec(c, op) != 0);
  }
  std::vector<char> in_tile(inst.size(), 0);
  Arena ar, at;
  for (int k = 0; k < n; ++k) {
    const int w = uses[k][2];
    if (w >= 0 && !inst[w].banned && inst[w].size <= cap) {
      const int64_t off = ar.alloc(inst[w].size);
      if (off + inst[w].size <= cap)
        inst[w].lds = base + off;
      else
        ar.release(off, inst[w].size);
    }
    if (w >= 0 && !inst[w].banned && inst[w].lds < 0 && inst[w].last > k && inst[w].size <= tcap &&
        tile_use[inst[w].last + 1] == tile_use[k]) {
      const int64_t off = at.alloc(inst[w].size);
      if (off + inst[w].size <= tcap) {
        inst[w].lds = tbase + off;
        in_tile[w] = 1;
      } else {
        at.release(off, inst[w].size);
      }
    }
    const DOp &op = (*c.ops)[ln.op_begin[v] + k];
    LdsOp &r = res[k];
    const bool thin = op.type == OP_CONTRACT && level_prec(c, op) == 0;
    if (thin || op.type == OP_LEAFGRAD) {
      const int64_t offs[2] = {op.x, op.y};
      for (int s = 0; s < (thin ? 2 : 1); ++s) {
        const int t = uses[k][s];
        const int32_t flag = s == 0 ? kLdsX : kLdsY;
        int64_t at = -1;
        if (offs[s] < leaf) at = mirror ? offs[s] : -1;
        else if (t >= 0) at = inst[t].lds;
        if (at >= 0) {
          r.flags |= flag;
          (s == 0 ? r.x : r.y) = (int32_t)at;
        }
      }
      if (thin && w >= 0 && inst[w].lds >= 0) {
        r.flags |= kLdsZ;
        r.z = (int32_t)inst[w].lds;
      }
      if (!thin && *acc_at >= 0 && op.y >= ln.gbar_begin && op.y + (int64_t(1) << op.nFX) <= ln.gbar_begin + ln.ptens_elems) {
        r.flags |= kLdsY;  // the accumulator
        r.y = (int32_t)(*acc_at + op.y - ln.gbar_begin);
      }
    }
    // give back what this op read for the last time, and a result nobody reads
    for (int s = 0; s < 3; ++s) {
      const int t = uses[k][s];
      if (t < 0 || inst[t].lds < 0) continue;
      if ((s < 2 && inst[t].last == k) || (s == 2 && inst[t].last < 0)) {
        if (in_tile[t])
          at.release(inst[t].lds - tbase, inst[t].size);
        else
          ar.release(inst[t].lds - base, inst[t].size);
        inst[t].lds = -2;  // released
      }
    }
  }
  return res;
}

// Summed-index bit positions of a thin op with nS <= kPackedTabBits, from
// its table (entry 2^t holds the offsets of summed bit t alone): 5 bits per
// position, lowest summed bit first.
static bool packed_tab(const ItemCtx &c, const DOp &op, int32_t &px, int32_t &py) {
  if (op.type != OP_CONTRACT || op.nS > kPackedTabBits || op.nS > kTabLoBits || !c.tabs) return false;
  px = py = 0;
  for (int t = 0; t < op.nS; ++t) {
    const int32_t ox = (*c.tabs)[op.tab + 2 * (1 << t)], oy = (*c.tabs)[op.tab + 2 * (1 << t) + 1];
    if (ox <= 0 || oy <= 0 || (ox & (ox - 1)) || (oy & (oy - 1))) return false;
    px |= (__builtin_ctz((uint32_t)ox) & 31) << (5 * t);
    py |= (__builtin_ctz((uint32_t)oy) & 31) << (5 * t);
  }
  return true;
}

// Bit positions of a matrix-core op's per-summed-bit offsets (the table
// entries of the single bits, as the tiles read them) into w[0..5] (X in
// w[0..2], Y in w[3..5], 5 bits each, six per word), when every one is a
// power of two and nS <= 18.
static bool mfma_packed_bits(const ItemCtx &c, const DOp &op, int32_t *w) {
  if (!c.tabs || op.nS > 18) return false;
  int32_t v[6] = {0, 0, 0, 0, 0, 0};
  const int lo = std::min(op.nS, kTabLoBits);
  for (int t = 0; t < op.nS; ++t) {
    const int64_t e = t < kTabLoBits ? (int64_t)2 << t : ((int64_t)2 << lo) + ((int64_t)2 << (t - kTabLoBits));
    const int32_t ox = (*c.tabs)[op.tab + e], oy = (*c.tabs)[op.tab + e + 1];
    if (ox <= 0 || oy <= 0 || (ox & (ox - 1)) || (oy & (oy - 1))) return false;
    v[t / 6] |= __builtin_ctz((uint32_t)ox) << (5 * (t % 6));
    v[3 + t / 6] |= __builtin_ctz((uint32_t)oy) << (5 * (t % 6));
  }
  std::copy(v, v + 6, w);
  return true;
}

// --- level items ------------------------------------------------------------------------------

// Runs of up to four consecutive record items whose contractions (or leaf
// adjoint additions) touch disjoint LDS ranges where one of them writes (no read-after-write,
// write-after-read or write-after-write between them) become one item: wave w
// runs the w-th (their records are consecutive), one barrier for all.
static void group_records(std::vector<PItem> &items, size_t first) {
  struct Rng {
    int64_t lo, hi;
  };
  auto ranges = [](const DOp &op, Rng &x, Rng &y, Rng &z) {
    x = {op.x, op.x + ((int64_t)1 << (op.nFX + op.nB + op.nS))};
    y = {op.y, op.y + ((int64_t)1 << (op.nS + op.nB + op.nFY))};
    z = {op.z, op.z + ((int64_t)1 << (op.nFX + op.nB + op.nFY))};
    if (op.type == OP_LEAFGRAD) y = z = {op.y, op.y + ((int64_t)1 << op.nFX)};  // adds into its accumulator
  };
  auto overlap = [](const Rng &a, const Rng &b) { return a.lo < b.hi && b.lo < a.hi; };
  std::vector<PItem> outv(items.begin(), items.begin() + first);
  for (size_t i = first; i < items.size();) {
    PItem head = items[i];
    size_t j = i + 1;
    if (head.kind == PK_TREC) {
      std::vector<std::array<Rng, 3>> grp(1);
      ranges(head.op, grp[0][0], grp[0][1], grp[0][2]);
      while (j < items.size() && grp.size() < 4 && items[j].kind == PK_TREC &&
             items[j].rec == head.rec + (int32_t)grp.size()) {
        std::array<Rng, 3> r;
        ranges(items[j].op, r[0], r[1], r[2]);
        bool ok = true;
        for (const auto &g : grp)
          ok = ok && !overlap(g[2], r[0]) && !overlap(g[2], r[1]) && !overlap(g[2], r[2]) && !overlap(r[2], g[0]) &&
               !overlap(r[2], g[1]);
        if (!ok) break;
        grp.push_back(r);
        ++j;
      }
      head.count = (int32_t)grp.size();
    }
    outv.push_back(head);
    i = j;
  }
  items.swap(outv);
}

// Runs of consecutive record items (after grouping) become one item of up
// to kMaxRunSteps steps: step t runs 1-4 records on waves 0.. (the counts,
// less one, packed 2 bits per step into a0 .. a5), lgl = the number of
// steps, count = the first step's count. Their records are consecutive.
static void run_records(std::vector<PItem> &items, size_t first) {
  std::vector<PItem> outv(items.begin(), items.begin() + first);
  for (size_t i = first; i < items.size();) {
    PItem head = items[i];
    size_t j = i + 1;
    if (head.kind == PK_TREC) {
      int32_t packed[6] = {0, 0, 0, 0, 0, 0};
      int steps = 0, next_rec = head.rec;
      for (j = i; j < items.size() && items[j].kind == PK_TREC && steps < kMaxRunSteps && items[j].rec == next_rec; ++j) {
        packed[steps >> 4] |= (items[j].count - 1) << (2 * (steps & 15));
        next_rec += items[j].count;
        ++steps;
      }
      head.lgl = steps;
      head.a0 = packed[0];
      head.a1 = packed[1];
      head.a2 = packed[2];
      head.a3 = packed[3];
      head.a4 = packed[4];
      head.a5 = packed[5];
    }
    outv.push_back(head);
    i = j;
  }
  items.swap(outv);
}

// Contraction shapes with a lane-record form: at most 64 outputs (summed
// index up to 12 bits), or an outer product of at most 256 outputs.
static bool record_shape(const DOp &op) {
  const int lgOut = op.nFX + op.nB + op.nFY;
  return op.type == OP_CONTRACT && ((lgOut <= 6 && op.nS <= 12) || (op.nS == 0 && lgOut <= 8));
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Items of one network's program variant v over n_sets parameter vectors:
// set-up, one item per op (two for a split matrix-core product or a rank-0
// contraction on several workgroups per vector), outputs.
void network_items(const ItemCtx &c, const LevelNet &ln, int v, int n_sets, int64_t abase, int64_t sbase,
                   int64_t pbase, int64_t zbase, bool allow_split, std::vector<PItem> &out, int64_t *split_need,
                   int64_t *part_need) {
  const int eb = c.dtype == TN_C128 ? 16 : 8;
  int lgs = 0;
  while ((int64_t(1) << lgs) < n_sets) ++lgs;
  auto base_item = [&](int kind) {
    PItem it{};
    it.rec = it.nrec = -1;
    it.nrec_n = 0;
    it.kind = kind;
    it.base = abase;
    it.stride = ln.stride[v];
    it.sbase = sbase;
    it.n_comp = std::max(1, ln.n_comp);
    return it;
  };
  const size_t first_item = out.size();
  auto push = [&](const PItem &it) { out.push_back(it); };
  int64_t acc_at = -1;
  const std::vector<LdsOp> lds = lds_assign(c, ln, v, &acc_at);
  {
    PItem it = base_item(PK_SETUP);
    it.mv = (lds_mirror(c, ln) ? 1 : 0) | (acc_at >= 0 ? 2 : 0);
    it.a4 = (int32_t)std::max<int64_t>(acc_at, 0);
    const int64_t zero_n = v == 1 ? ln.ptens_elems : 0;
    const int64_t per = ln.n_const + ln.ptens_elems + zero_n;
    it.lgl = c.one_wg ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(64, ceil_div(per, 1024)));
    it.count = it.lgl * n_sets;
    it.a0 = ln.const_begin;
    it.a1 = ln.n_const;
    it.a2 = ln.ptens_begin;
    it.a3 = ln.n_ptens;
    it.zs = ln.gbar_begin;
    it.a5 = (int32_t)zero_n;
    push(it);
  }
  for (int k = 0; k < ln.n_ops[v]; ++k) {
    const DOp &op = (*c.ops)[ln.op_begin[v] + k];
    PItem it = base_item(PK_THIN);
    it.op = op;
    pack_runs(op.maskX, it.ru.runsX);
    pack_runs(op.maskY, it.ru.runsY);
    const int prec = op.type == OP_CONTRACT ? level_prec(c, op) : 0;
    if (prec) {
      it.kind = PK_MFMA;
      const int shape = level_tile(c, op);
      it.mv = mfma_variant(op, prec, shape);
      if (mfma_packed_bits(c, op, &it.a0)) it.mv |= kMfmaPacked;
      const int64_t wg = (int64_t)mfma_tiles(op, shape) * n_sets;
      const int64_t part = (int64_t)n_sets << (op.nFX + op.nFY);  // elements per range
      int ls = 0;
      while (allow_split && ls < 6 && op.nS - ls > 9 && (wg << ls) < c.split_target &&
             (part << (ls + 1)) * eb <= kSplitItemBytes)
        ++ls;
      it.lgl = ls;
      it.count = (int32_t)(wg << ls);
      it.zs = zbase;
      push(it);
      if (ls > 0) {
        *split_need = std::max(*split_need, part << ls);
        PItem r = base_item(PK_SPLITSUM);
        r.op = op;
        r.lgl = ls;
        r.zs = zbase;
        r.count = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kItemMaxTasks, ceil_div(part, 256)));
        push(r);
      }
    } else if (op.type == OP_CONTRACT || op.type == OP_LEAFGRAD) {
      const bool thin = op.type == OP_CONTRACT;
      if (c.one_wg) {
        const LdsOp &r = lds[k];
        it.a0 = r.flags;
        if (r.flags & kLdsX) it.op.x = r.x;
        if (r.flags & kLdsY) it.op.y = r.y;
        if (r.flags & kLdsZ) it.op.z = r.z;
        if (thin && packed_tab(c, op, it.a1, it.a2)) it.a0 |= kPackedTab;
        // a small contraction with every operand in LDS: one wave runs it
        // from a lane record (offsets precomputed here). Measured: with an
        // operand in the region the vector-unit path is faster.
        if (thin && c.trecs && (r.flags & (kLdsX | kLdsY | kLdsZ)) == (kLdsX | kLdsY | kLdsZ) &&
            record_shape(it.op)) {
          const size_t at = c.trecs->size();
          const int type = build_record(*c.tabs, {}, it.op, *c.trecs);
          if (type == kRecLite || type == kRecWide || type == kRecNarrow) {
            it.kind = PK_TREC;
            it.rec = (int32_t)(at / (4 * kRecLanes));
            it.count = 1;
          } else {
            c.trecs->resize(at);
          }
        }
        // a leaf adjoint with its adjoint and accumulator in LDS: one wave
        // adds it from a record
        if (!thin && c.trecs && (r.flags & (kLdsX | kLdsY)) == (kLdsX | kLdsY) && op.nFX <= 8 &&
            it.op.y < (1 << 17)) {
          it.kind = PK_TREC;
          it.rec = (int32_t)(c.trecs->size() / (4 * kRecLanes));
          it.count = 1;
          for (int l = 0; l < kRecLanes; ++l) {
            int32_t cy = 0;
            for (int q = 0; q < 4; ++q)
              if (l + (q << 6) < (1 << op.nFX)) cy |= ((*c.tabs)[op.tab + l + (q << 6)] & 0xff) << (8 * q);
            c.trecs->push_back((int32_t)it.op.x + l);
            c.trecs->push_back(cy);
            c.trecs->push_back(0);
            c.trecs->push_back(l == 0 ? (int32_t)(kRecAcc | (op.nFX << 7) | ((uint32_t)it.op.y << 15)) : 0);
          }
        }
      }
      const int lg = thin ? op.nFX + op.nB + op.nFY : op.nFX;
      int64_t work = ((int64_t)1 << lg) * n_sets;
      it.lgl = 0;
      if (thin) {
        // lanes per output: at least 8 summed entries each, up to 64, while
        // the step has fewer than 2^20 (output, lane) pairs (one workgroup:
        // at least 2 entries each and 2^8 pairs, one per thread; measured
        // against 1 .. 16 entries and 2^6 .. 2^11 pairs)
        const int lg_fill = c.one_wg ? 8 : 20, lg_four = c.one_wg ? 10 : 16;
        it.lgl = std::max(0, std::min({6, op.nS - (c.one_wg ? 1 : 3), lg_fill - lg - lgs}));
        work <<= it.lgl;
        // many outputs: four per lane instead (shared operand reads)
        if (it.lgl == 0 && lg + lgs >= lg_four && (op.nFY >= 2 || (op.nFY == 0 && op.nB == 0 && op.nFX >= 8))) {
          // 64 apart along Y (>= 8 Y-only bits) or X (X-only output bits), else consecutive
          it.lgl = op.nFY >= 8 ? -2 : op.nFY == 0 ? -3 : -1;
          work >>= 2;
        }
      }
      it.count = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kItemMaxTasks, ceil_div(work, 256)));
      push(it);
    } else if (op.type == OP_SCALAR) {
      it.kind = PK_SCALAR;
      const int64_t K = (int64_t)1 << op.nS;
      const int G = c.one_wg ? 1 : (int)std::min<int64_t>(kScalarParts, std::max<int64_t>(1, K / 1024));
      it.lgl = G;
      it.count = G * n_sets;
      it.zs = pbase;
      push(it);
      if (G > 1) {
        *part_need = std::max(*part_need, (int64_t)n_sets * G * 2);
        PItem r = base_item(PK_SCALAR_SUM);
        r.op = op;
        r.a0 = G;
        r.zs = pbase;
        r.count = (int32_t)ceil_div(n_sets, 256);
        push(r);
      }
    } else {  // OP_SEED
      it.kind = PK_SEED;
      it.count = (int32_t)ceil_div(n_sets, 256);
      push(it);
    }
  }
  PItem f = base_item(PK_FINISH);
  f.count = n_sets;
  f.a0 = ln.net;
  f.a1 = ln.ptens_begin;
  f.a2 = ln.n_ptens;
  f.mv = acc_at >= 0 ? 1 : 0;  // adjoint accumulators in LDS from a3
  f.a3 = (int32_t)std::max<int64_t>(acc_at, 0);
  f.zs = ln.gbar_begin;
  push(f);
  if (c.one_wg) {
    group_records(out, first_item);
    run_records(out, first_item);
  }
  for (size_t i = first_item; i + 1 < out.size(); ++i) {
    out[i].nrec = out[i + 1].rec;
    out[i].nrec_n = out[i + 1].kind == PK_TREC ? out[i + 1].count : 0;
  }
}

// Items of every group (item mode) or its task-executor items and networks,
// and the items of the networks run alone, for the current matrix-core
// choices.
int plan_level(tn_batch *b) {
  b->trecs.clear();
  for (int v = 0; v < 2; ++v) {
    b->items[v].clear();
    b->titems[v].clear();
    b->tnets[v].clear();
    b->solo_items[v].clear();
    b->solo_begin[v].clear();
    for (LevelGroup &g : b->groups) {
      g.item0[v] = (int)b->items[v].size();
      g.tasked = (int64_t)g.lv.size() * b->max_sets >= b->task_min;
      g.tnet0 = (int)b->tnets[v].size();
      if (!g.tasked) {
        for (size_t j = 0; j < g.lv.size(); ++j) {
          int64_t sn = 0, pn = 0;
          const size_t at = b->items[v].size();
          network_items(item_ctx(b), b->level[g.lv[j]], v, b->max_sets, g.abase[j], g.sbase[j], g.pbase[j],
                        g.zbase[j], true, b->items[v], &sn, &pn);
          if (sn > g.zsize[j]) {  // more split scratch than planned: no split sums for this network
            b->items[v].resize(at);
            network_items(item_ctx(b), b->level[g.lv[j]], v, b->max_sets, g.abase[j], g.sbase[j], g.pbase[j],
                          g.zbase[j], false, b->items[v], &sn, &pn);
          }
        }
        g.n_items[v] = (int)b->items[v].size() - g.item0[v];
        continue;
      }
      g.n_items[v] = 0;
      // networks by decreasing cost: their tasks are taken first
      std::vector<int> order(g.lv.size());
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(),
                       [&](int x, int y) { return b->level[g.lv[x]].cost > b->level[g.lv[y]].cost; });
      ItemCtx c = item_ctx(b);
      c.one_wg = true;
      // every eligible product on the matrix cores: the tuner's per-class
      // choices are timed on chip-wide item launches, not on one workgroup
      c.use_mfma = nullptr;
      c.lds_elems = b->dtype == TN_C128 ? kLdsArenaBytes<TN_MFMA_FP64> / 16 : kLdsArenaBytes<TN_MFMA_FP32> / 8;
      {
        const int tb = b->dtype == TN_C128 ? kTileLdsBytes<TN_MFMA_FP64>
                       : b->mfma_prec == TN_MFMA_BF16X3 ? kTileLdsBytes<TN_MFMA_BF16X3> : kTileLdsBytes<TN_MFMA_FP32>;
        c.tile_elems = (tb - kTileReserve) / (b->dtype == TN_C128 ? 16 : 8);
      }
      if (const char *env = std::getenv("QTN_TASK_LDS")) {
        c.lds_elems = std::min(c.lds_elems, std::max(0, std::atoi(env)));
        if (c.lds_elems == 0) c.tile_elems = 0;
      }
      c.trecs = &b->trecs;
      for (int j : order) {
        const LevelNet &ln = b->level[g.lv[j]];
        TNet tn{};
        tn.abase = g.abase[j];
        tn.stride = ln.stride[v];
        tn.sbase = g.sbase[j];
        tn.n_comp = std::max(1, ln.n_comp);
        tn.item0 = (int)b->titems[v].size();
        int64_t sn = 0, pn = 0;
        network_items(c, ln, v, 1, 0, 0, 0, 0, false, b->titems[v], &sn, &pn);
        tn.n_items = (int)b->titems[v].size() - tn.item0;
        b->tnets[v].push_back(tn);
      }
    }
    for (int l : b->lsolo) {
      const LevelNet &ln = b->level[l];
      int64_t sn = 0, pn = 0;
      b->solo_begin[v].push_back((int)b->solo_items[v].size());
      network_items(item_ctx(b), ln, v, ln.chunk, 0, 0, 0, 0, false, b->solo_items[v], &sn, &pn);
    }
    b->solo_begin[v].push_back((int)b->solo_items[v].size());
  }
  b->items_dirty = true;
  return TN_OK;
}

// Task-executor items of one network: one per op plus set-up and outputs,
// whatever runs each product (no split or partial-sum items).
static int64_t titem_count(const LevelNet &ln, int v) { return (int64_t)ln.n_ops[v] + 2; }

// Device workspace: byte offsets of every array (256-byte aligned).
void plan_workspace(tn_batch *b) {
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const HostProgram &hp = b->hp;
  b->cap_titems[0] = b->cap_titems[1] = 0;
  int64_t n_tnets = 0;
  b->cap_trecs = 0;
  for (const LevelGroup &g : b->groups) {
    n_tnets += (int64_t)g.lv.size();
    for (int v = 0; v < 2; ++v)
      for (int l : g.lv) {
        b->cap_titems[v] += titem_count(b->level[l], v);
        const LevelNet &ln = b->level[l];
        for (int k = 0; k < ln.n_ops[v]; ++k) {
          const DOp &op = hp.ops[ln.op_begin[v] + k];
          b->cap_trecs += record_shape(op) || (op.type == OP_LEAFGRAD && op.nFX <= 8) ? 4 * kRecLanes : 0;
        }
      }
  }
  WsLayout &w = b->ws;
  auto sz = [&](int k, int64_t bytes) { w.size[k] = std::max<int64_t>(bytes, 0); };
  sz(WsLayout::NETS_FWD, hp.nets_fwd.size() * sizeof(DNet));
  sz(WsLayout::NETS_GRAD, hp.nets_grad.size() * sizeof(DNet));
  sz(WsLayout::OPS, hp.ops.size() * sizeof(DOp));
  sz(WsLayout::TABS, hp.tabs.size() * sizeof(int32_t));
  sz(WsLayout::RECS, hp.recs.size() * sizeof(int32_t));
  sz(WsLayout::SRECS0, hp.srecs[0].size() * sizeof(int32_t));
  sz(WsLayout::SRECS1, hp.srecs[1].size() * sizeof(int32_t));
  sz(WsLayout::TASK_NET, b->task_net.size() * sizeof(int32_t));
  sz(WsLayout::GTASK_NET, b->gtask_net.size() * sizeof(int32_t));
  sz(WsLayout::CONSTS, (int64_t)(hp.consts.size() / 2) * eb);
  sz(WsLayout::PTENS, hp.ptens.size() * sizeof(DParam));
  sz(WsLayout::SLOTS, hp.slots.size() * sizeof(DParam));
  sz(WsLayout::COEF, (int64_t)b->n_nets * 8);
  sz(WsLayout::BOUND, (int64_t)b->max_sets * std::max(1, hp.per_set) * eb);
  sz(WsLayout::DBOUND, (int64_t)b->max_sets * std::max(1, hp.per_set) * eb);
  sz(WsLayout::VAL, (int64_t)b->n_nets * b->max_sets * 2 * 8);
  sz(WsLayout::GNET, (int64_t)b->n_nets * b->max_sets * std::max(1, b->n_params) * 8);
  sz(WsLayout::GARENA, b->gtask_net.empty() ? 0 : (int64_t)b->gslots * b->gstride * eb);
  sz(WsLayout::LARENA, b->larena_elems * eb);
  sz(WsLayout::LSCAL, b->lscal_doubles * 8);
  sz(WsLayout::LPART, b->lpart_doubles * 8);
  sz(WsLayout::LSPLIT, b->lsplit_elems * eb);
  sz(WsLayout::TITEMS0, b->cap_titems[0] * (int64_t)sizeof(PItem));
  sz(WsLayout::TITEMS1, b->cap_titems[1] * (int64_t)sizeof(PItem));
  sz(WsLayout::TNETS0, n_tnets * (int64_t)sizeof(TNet));
  sz(WsLayout::TNETS1, n_tnets * (int64_t)sizeof(TNet));
  sz(WsLayout::TRECS, b->cap_trecs * (int64_t)sizeof(int32_t));
  sz(WsLayout::CTRL, 64);
  int64_t off = 0;
  for (int k = 0; k < WsLayout::N; ++k) {
    w.off[k] = off;
    off += (std::max<int64_t>(w.size[k], 1) + 255) & ~int64_t(255);
  }
  w.total = off;
}

// Host part of tn_batch_create: programs, executors, level groups, items and
// the workspace layout. No GPU calls.
int plan_batch(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch *b) {
  if (!nets || n_nets < 1 || max_sets < 1) {
    set_error("tn_batch_create: bad arguments");
    return TN_EINVAL;
  }
  const Net *n0 = reinterpret_cast<const Net *>(nets[0]);
  for (int i = 0; i < n_nets; ++i) {
    const Net *n = reinterpret_cast<const Net *>(nets[i]);
    if (!n) { set_error("tn_batch_create: NULL network"); return TN_EINVAL; }
    if (!n->has_order) { set_error("tn_batch_create: network " + std::to_string(i) + " has no order"); return TN_EORDER; }
    if (n->poisoned) { set_error("tn_batch_create: network poisoned"); return TN_ESTATE; }
    if (n->dtype != n0->dtype || n->n_params != n0->n_params) {
      set_error("tn_batch_create: networks differ in dtype or n_params");
      return TN_EINVAL;
    }
  }
  b->dtype = n0->dtype;
  b->mfma_prec = b->dtype == TN_C128 ? TN_MFMA_FP64 : TN_MFMA_FP32;
  b->n_nets = n_nets;
  b->n_params = n0->n_params;
  b->max_sets = max_sets;
  b->offset = offset;
  b->coef.assign(n_nets, 0.0);
  if (coef) std::copy(coef, coef + n_nets, b->coef.begin());
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  // QTN_FUSED_LDS_MAX (bytes) overrides the LDS-fused limit, e.g. 0 sends
  // every network to the global-arena or level executor
  int64_t fused_max = kFusedLdsMax;
  const char *fused_env = std::getenv("QTN_FUSED_LDS_MAX");
  const bool fused_max_set = fused_env != nullptr;
  if (fused_env) fused_max = std::atoll(fused_env);
  int64_t gmem_max = kGmemMaxMacs;  // QTN_GMEM_MAX_MACS=0 turns the global-arena executor off
  if (const char *env = std::getenv("QTN_GMEM_MAX_MACS")) gmem_max = std::atoll(env);
  int64_t level_budget = kLevelBudget;  // QTN_LEVEL_BUDGET (bytes): level arena limit
  if (const char *env = std::getenv("QTN_LEVEL_BUDGET")) level_budget = std::max<int64_t>(1, std::atoll(env));
  b->split_target = kSplitTarget;  // QTN_SPLIT_TARGET=0 keeps every matrix-core sum on one task
  if (const char *env = std::getenv("QTN_SPLIT_TARGET")) b->split_target = std::max<int64_t>(0, std::atoll(env));
  if (const char *env = std::getenv("QTN_TASK_MIN")) b->task_min = std::max(1, std::atoi(env));
  std::vector<double> cost(n_nets);
  std::vector<int> fused_ids, gmem_ids;
  int maxbits = 0;
  // executor of each network: the LDS fused executor when its memory fits
  // LDS, the global-arena fused executor when its steps are small enough for
  // one workgroup, else the level executor. The global-arena networks join
  // the level ones on the task executor (one launch, LDS-resident small
  // tensors, matrix cores for the few large steps) when the level networks
  // are enough for it anyway (measured faster on the 5-regular p=2 batches),
  // or when the global-arena ones are enough for it and hold at least
  // kGmemJoinMacs multiply-adds per parameter vector in all (measured on the
  // p=2 batches: 4-regular n=70 and n=100 6.4 -> 3.1 and 6.7 -> 4.1 ms, the
  // 5-regular n=50 diagonal one 5.1 -> 3.8 ms; below it the global-arena
  // executor stayed faster, e.g. 4.0 against 5.6 ms on the 5-regular n=100
  // diagonal batch, 3.4e6 multiply-adds).
  struct Classes {
    std::vector<int> cls;
    int n_level = 0, n_gmem = 0;
    double gmem_macs = 0;  // multiply-adds of the global-arena networks, one parameter vector
  };
  auto classify = [&](int64_t fmax) {
    Classes k;
    k.cls.resize(n_nets);
    for (int i = 0; i < n_nets; ++i) {
      const Net *n = reinterpret_cast<const Net *>(nets[i]);
      NetLayout lay = make_layout(*n);
      double max_macs = 0, tot_macs = 0;
      for (const Op &op : n->gplan.ops)
        if (op.type == OP_CONTRACT || op.type == OP_SCALAR) {
          const double m = std::ldexp(1.0, op.nFX + op.nB + op.nS + op.nFY);
          max_macs = std::max(max_macs, m);
          tot_macs += m;
        }
      const int64_t mem_elems = lay.leaf_region + std::max(lay.arena[0], lay.arena[1]);
      int &c = k.cls[i];
      if (fused_lds_need(*n, lay, eb, b->n_params) <= fmax)
        c = 0;
      else if (tot_macs <= (double)gmem_max && max_macs <= (double)gmem_max / 16 && mem_elems < kMaxArenaElems &&
               mem_elems * eb <= kGmemBudget / 256)
        c = 2;
      else
        c = 1;
      k.n_level += c == 1;
      k.n_gmem += c == 2;
      if (c == 2) k.gmem_macs += tot_macs;
    }
    return k;
  };
  bool join = true;  // QTN_GMEM_JOIN=0 keeps them on the global-arena executor
  if (const char *env = std::getenv("QTN_GMEM_JOIN")) join = std::atoi(env) != 0;
  // the global-arena networks join the task executor because the level ones are enough
  // for it (1), or because they hold enough work themselves (2)
  auto joins = [&](const Classes &k) {
    if (!join || k.n_gmem == 0) return 0;
    if ((int64_t)k.n_level * max_sets >= b->task_min) return 1;
    return (int64_t)k.n_gmem * max_sets >= b->task_min && k.gmem_macs >= kGmemJoinMacs ? 2 : 0;
  };
  Classes k = classify(fused_max);
  // Networks between the fused limit and kFusedLdsMaxHi stay on the fused
  // executor when moving them only sends light global-arena networks to the
  // task executor (measured: the 5-regular n=100 p=2 diagonal batch 5.4 ms
  // with them moved, 4.1 ms kept; the batches whose networks move to the
  // level or global-arena executor otherwise run faster moved)
  if (!fused_max_set && fused_max < kFusedLdsMaxHi && joins(k) == 2) {
    Classes hi = classify(kFusedLdsMaxHi);
    if (joins(hi) == 0) k = std::move(hi);
  }
  std::vector<int> &cls = k.cls;
  if (joins(k))
    for (int &c : cls)
      if (c == 2) c = 1;
  for (int i = 0; i < n_nets; ++i) {
    const Net *n = reinterpret_cast<const Net *>(nets[i]);
    NetLayout lay = make_layout(*n);
    cost[i] = n->gplan.flops + n->gplan.flops_grad + 1e3 * n->gplan.ops.size();
    int ex = -1;  // executor: 0 LDS fused, 1 level, 2 global arena
    b->flops_fwd += n->gplan.flops;
    b->bytes_fwd += n->gplan.bytes;
    b->flops_grad += n->gplan.flops_grad;
    b->bytes_grad += n->gplan.bytes_grad;
    if (cls[i] == 0) {
      append_fused(*n, lay, b->hp, false);
      fused_ids.push_back(i);
      ex = 0;
      maxbits = std::max(maxbits, n->gplan.peak_bits);
    } else if (cls[i] == 2) {
      append_fused(*n, lay, b->hp, true);
      gmem_ids.push_back(i);
      ex = 2;
    } else {
      b->hp.nets_fwd.push_back(DNet{});
      b->hp.nets_grad.push_back(DNet{});
      b->level.push_back(append_level(*n, lay, b->hp, i, eb, level_budget, max_sets));
      ex = 1;
      if (b->level.back().stride[0] >= kMaxLevelElems) {
        set_error("tn_batch_create: network " + std::to_string(i) + " needs " +
                  std::to_string(b->level.back().stride[0]) +
                  " elements of working memory per parameter vector; the executor addresses at most 2^40");
        return TN_ENOMEM;
      }
    }
    b->exec_flops[ex] += n->gplan.flops + n->gplan.flops_grad;
    b->exec_bytes[ex] += n->gplan.bytes + n->gplan.bytes_grad;
  }
  // fused networks, expensive first (longest processing time first)
  b->task_net = fused_ids;
  std::stable_sort(b->task_net.begin(), b->task_net.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  b->gtask_net = gmem_ids;
  std::stable_sort(b->gtask_net.begin(), b->gtask_net.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  // block size: enough threads for the typical op, few idle lanes
  b->block = maxbits <= 6 ? 64 : (maxbits <= 9 ? 128 : 256);
  if (const char *env = std::getenv("QTN_FUSED_BLOCK")) {
    int v = std::atoi(env);
    if (v == 64 || v == 128 || v == 256) b->block = v;
  }
  // several angle sets per wave when every op has a set-packed record and
  // their memory stays within the fused budget. Measured default: four for
  // forward programs (many small steps), one for adjoint programs (their
  // larger LDS need leaves too few waves to hide latency). QTN_SETS_PER_WAVE
  // (1, 2, 4) asks for a count for both; the autotuner compares them.
  b->fused_budget = fused_max;
  int want[2] = {4, 1};
  if (const char *env = std::getenv("QTN_SETS_PER_WAVE")) want[0] = want[1] = std::atoi(env);
  if (max_sets == 1) want[0] = want[1] = 1;  // one angle set: nothing to pack
  for (int v = 0; v < 2; ++v) {
    if (want[v] == 4 && sets_fit(b, 4, fused_max, v)) b->spw[v] = 4;
    else if (want[v] >= 2 && sets_fit(b, 2, fused_max, v)) b->spw[v] = 2;
  }
  // global-arena slots: one per resident workgroup, within the budget
  if (!b->gtask_net.empty()) {
    b->gstride = (std::max(b->hp.max_mem_g[0], b->hp.max_mem_g[1]) + 63) & ~int64_t(63);
    // no more slots than tasks: a launch never runs more workgroups
    const int64_t tasks = (int64_t)b->gtask_net.size() * max_sets;
    b->gslots = (int)std::max<int64_t>(1, std::min<int64_t>({2048, kGmemBudget / (b->gstride * eb), tasks}));
  }
  // groups: level networks that take every parameter vector at once, packed
  // in order while their regions fit the level budget together
  int64_t arena = 0, scal = 0, part = 0, split = 0;
  int64_t g_elems = 0, g_scal = 0, g_part = 0, g_split = 0;
  for (int l = 0; l < (int)b->level.size(); ++l) {
    const LevelNet &ln = b->level[l];
    const int64_t per = ln.stride[ln.grad_ok ? 1 : 0];
    if (ln.chunk < max_sets) {
      b->lsolo.push_back(l);
      arena = std::max(arena, per * ln.chunk);
      scal = std::max(scal, (int64_t)ln.chunk * std::max(1, ln.n_comp) * 2);
      part = std::max(part, (int64_t)ln.chunk * kScalarParts * 2);
      continue;
    }
    // this network's rank-0 partial sums and split partial tiles, both variants
    int64_t sn = 0, pn = 0;
    for (int v = 0; v < 2; ++v)
      for (int shape = 0; shape < 4; ++shape) {  // whichever tile shape the tuner picks
        std::vector<PItem> tmp;
        ItemCtx c = item_ctx(b);
        c.use_mfma = nullptr;  // every eligible op on the matrix cores: the most scratch
        c.force_tile = shape;
        network_items(c, ln, v, max_sets, 0, 0, 0, 0, true, tmp, &sn, &pn);
      }
    const int64_t need = (per * max_sets + 63) / 64 * 64;
    if (b->groups.empty() || (g_elems + need) * eb > level_budget) {
      b->groups.emplace_back();
      g_elems = g_scal = g_part = g_split = 0;
    }
    LevelGroup &g = b->groups.back();
    g.lv.push_back(l);
    g.abase.push_back(g_elems);
    g.sbase.push_back(g_scal);
    g.pbase.push_back(g_part);
    g.zbase.push_back(g_split);
    g.zsize.push_back(sn);
    g_elems += need;
    g_scal += (int64_t)max_sets * std::max(1, ln.n_comp) * 2;
    g_part += pn;
    g_split += (sn + 63) / 64 * 64;
    arena = std::max(arena, g_elems);
    scal = std::max(scal, g_scal);
    part = std::max(part, g_part);
    split = std::max(split, g_split);
  }
  b->larena_elems = arena;
  b->lscal_doubles = scal;
  b->lpart_doubles = part;
  b->lsplit_elems = split;
  b->level_bytes = arena * eb;
  if (b->dtype == TN_C64) b->consts_f.assign(b->hp.consts.begin(), b->hp.consts.end());
  int rc = plan_level(b);
  if (rc != TN_OK) return rc;
  plan_workspace(b);
  return TN_OK;
}

int batch_create(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch **out) {
  if (!out) {
    set_error("tn_batch_create: out is NULL");
    return TN_EINVAL;
  }
  std::unique_ptr<tn_batch> b(new tn_batch());
  int rc = plan_batch(nets, n_nets, coef, offset, max_sets, b.get());
  if (rc != TN_OK) return rc;
  *out = b.release();
  return TN_OK;
}

// LDS bytes of the set-packed layout with S sets per wave: per set its
// memory, component scalars and gradient sums. The sets' regions start 64
// bytes apart modulo the 256-byte bank cycle, so the same lane of different
// sets reads different banks.
int set_lds_layout(const tn_batch *b, int S, int variant, int *stride, int *scal_off, int *gacc_off) {
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const int mem = variant == 0 ? b->hp.max_mem_fwd : b->hp.max_mem_grad;
  auto al = [](int x) { return (x + 15) & ~15; };
  const int unit = 256 / eb, shift = 64 / eb;
  const int base = (mem + 1) & ~1;
  *stride = base + ((shift - base % unit) % unit + unit) % unit;
  int o = al(S * *stride * eb);
  *scal_off = o;
  o = al(o + S * std::max(1, b->hp.max_comp) * 16);
  *gacc_off = o;
  return al(o + S * std::max(1, b->n_params) * 8);
}

// Set-packed form with S sets per wave available for a program variant and
// within the fused LDS budget.
bool sets_fit(const tn_batch *b, int S, int64_t budget, int variant) {
  if (b->task_net.empty() || !b->hp.sets_ok[S == 4 ? 0 : 1]) return false;
  int st, so, go;
  return set_lds_layout(b, S, variant, &st, &so, &go) <= std::min<int64_t>(budget, 64 * 1024);
}

int64_t batch_workspace_bytes(const tn_batch *b) { return b->ws.total; }

int plan_set_precision(tn_batch *b, int prec) {
  const bool ok = b->dtype == TN_C128 ? prec == TN_MFMA_FP64 : (prec == TN_MFMA_FP32 || prec == TN_MFMA_BF16X3);
  if (!ok) {
    set_error("tn_batch_set_precision: precision not available for this batch's dtype");
    return TN_EINVAL;
  }
  b->mfma_prec = prec;
  return plan_level(b);
}

int batch_info(const tn_batch *b, tn_batch_stats *s) {
  std::memset(s, 0, sizeof(*s));
  s->n_nets = b->n_nets;
  s->n_fused = (int32_t)b->task_net.size();
  s->n_global = (int32_t)b->gtask_net.size();
  s->n_level = (int32_t)b->level.size();
  int levels = 0;
  for (auto &ln : b->level) levels = std::max(levels, ln.n_ops[1]);
  s->n_levels = levels;
  s->n_level_groups = (int32_t)b->groups.size();
  for (const LevelGroup &g : b->groups) s->n_level_tasked += g.tasked;
  s->n_level_chunked = (int32_t)b->lsolo.size();
  for (int v = 0; v < 2; ++v) {
    // per group: counter reset and the task executor, or one launch per item
    int64_t n = 0;
    for (const LevelGroup &g : b->groups) n += g.tasked ? 2 : g.n_items[v];
    for (size_t q = 0; q < b->lsolo.size(); ++q) {
      const LevelNet &ln = b->level[b->lsolo[q]];
      n += (int64_t)(b->solo_begin[v][q + 1] - b->solo_begin[v][q]) * ((b->max_sets + ln.chunk - 1) / ln.chunk);
    }
    (v == 0 ? s->level_launches_fwd : s->level_launches_grad) = (int32_t)std::min<int64_t>(n, INT32_MAX);
    int32_t ns = 0;
    for (const PItem &it : b->items[v]) ns += it.kind == PK_SPLITSUM;
    (v == 0 ? s->level_split_fwd : s->level_split_grad) = ns;
  }
  s->n_programs = b->hp.n_programs;
  s->fused_block = b->block;
  s->sets_per_wave_fwd = b->spw[0];
  s->sets_per_wave_grad = b->spw[1];
  s->rec_only = (b->block == kRecLanes && !b->hp.generic[0] ? 1 : 0) | (b->block == kRecLanes && !b->hp.generic[1] ? 2 : 0);
  s->lds_bytes_fwd = b->lds_fwd;
  s->lds_bytes_grad = b->lds_grad;
  for (int x = 0; x < 3; ++x) {
    s->exec_flops[x] = b->exec_flops[x];
    s->exec_bytes[x] = b->exec_bytes[x];
  }
  // level ops on the matrix cores with the current choices (forward + adjoint)
  for (const LevelNet &ln : b->level)
    for (int k = 0; k < ln.n_ops[1]; ++k) {
      const DOp &op = b->hp.ops[ln.op_begin[1] + k];
      if (op.type == OP_CONTRACT && level_prec(b, op) != 0)
        s->level_mfma_flops += 8.0 * std::ldexp(1.0, op.nFX + op.nB + op.nS + op.nFY);
    }
  s->flops_fwd = b->flops_fwd;
  s->bytes_fwd = b->bytes_fwd;
  s->flops_grad = b->flops_grad;
  s->bytes_grad = b->bytes_grad;
  return TN_OK;
}

}  // namespace qtn
