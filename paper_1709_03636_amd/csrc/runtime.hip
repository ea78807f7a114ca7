// Batch runtime: turns compiled network programs into device arrays, lays
// out executor memory, launches the kernels and captures HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <array>
#include <cstring>
#include <functional>
#include <memory>
#include <map>
#include <numeric>
#include <tuple>

#include "device.hpp"
#include "internal.hpp"

namespace qtn {

hipError_t launch_fused_sets(int dtype, bool grad, int sets, const FusedArgs &a, int grid, int lds_bytes, hipStream_t st);
const void *fused_sets_kernel_ptr(int dtype, bool grad, int sets);
hipError_t launch_fused(int dtype, int block, bool grad, bool rec_only, bool gmem, const FusedArgs &a, int grid, int lds_bytes,
                        hipStream_t st);
const void *fused_kernel_ptr(int dtype, int block, bool grad, bool rec_only, bool gmem);
hipError_t launch_combine(const double *val, const double *gnet, const double *coef, double offset, int n_nets,
                          int n_sets, int n_params, double *obj, double *grad, hipStream_t st);
hipError_t launch_bind(int dtype, const DParam *slots, int n_slots, const double *params, int n_params, int n_sets,
                       int per_set, void *G, void *dG, hipStream_t st);
hipError_t level_op(int dtype, const LevelArgs &a, const DOp &op, const int32_t *tabs, int mfma, hipStream_t st);
hipError_t level_group(int dtype, const LItem *items, const int32_t *blk, int n, int blocks, void *arena, int n_sets,
                       const int32_t *tabs, hipStream_t st);
bool mfma_eligible(int dtype, const DOp &op);
hipError_t mfma_contract(const LevelArgs &a, const DOp &op, const int32_t *tab, int prec, hipStream_t st);
int mfma_tiles(const DOp &op);
int mfma_variant(const DOp &op, int prec);
hipError_t mfma_group(int variant, const LItem *items, const int32_t *blk, int n, int blocks, void *arena,
                      void *split, int n_sets, const int32_t *tabs, hipStream_t st);
hipError_t mfma_split_reduce(int dtype, const LItem *items, const int32_t *blk, int n, int blocks, void *arena,
                             const void *split, int n_sets, hipStream_t st);
hipError_t level_setup(int dtype, const LevelArgs &a, const void *consts, int n_const, const DParam *pt, int n_pt,
                       const void *bound, int per_set, int set0, int zero_begin, int zero_n, hipStream_t st);
hipError_t level_finish(int dtype, const LevelArgs &a, const DParam *pt, int n_pt, const void *dbound, int per_set,
                        int set0, int net, int n_sets_total, int n_params, double *out_val, double *out_grad,
                        int with_grad, hipStream_t st);


static constexpr int kLdsCap = 160 * 1024;
// Networks whose fused adjoint program needs more LDS than this run on the
// global-arena or level executor, so one large network does not lower the
// occupancy of all: at most 48 KiB keeps three workgroups per CU (a p=2
// 3-regular batch with 40-56 KiB programs ran 1.8x faster on HBM arena
// slots with more workgroups in flight than in LDS with two).
static constexpr int64_t kFusedLdsMax = 48 * 1024;
// Global-memory arena budget of the level executor: networks stepped
// together share it (more of them per group, fewer groups stepped one after
// another); a network alone processes its parameter vectors in chunks that
// fit. 32 GiB of the 288 GB of HBM.
static constexpr int64_t kLevelBudget = 32ll << 30;
static constexpr int64_t kMaxArenaElems = int64_t(1) << 31;  // 32-bit element offsets per set
// Global-arena fused executor: networks too large for LDS whose whole task
// (forward + adjoint program of one parameter vector) has at most this many
// complex multiply-adds, and no step above a sixteenth of it, run one
// workgroup per task. Heavier tasks need whole-GPU launches per step (level
// executor, matrix cores): one workgroup would serialise them.
static constexpr int64_t kGmemMaxMacs = int64_t(1) << 20;
static constexpr int64_t kGmemBudget = 16ll << 30;  // bytes of arena slots

// First-fit arena allocator over element offsets.
struct Arena {
  std::vector<std::pair<int64_t, int64_t>> free_;  // (offset, size), sorted by offset
  int64_t top = 0;
  int64_t alloc(int64_t n) {
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
  void release(int64_t off, int64_t n) {
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
};

// Offsets of the buffers >= n_leaves of ops [0, n_ops) by liveness.
static int64_t layout_buffers(const Plan &p, int n_ops, std::vector<int64_t> &off) {
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

// Layout of one network's buffers in executor memory: constant leaves,
// parametric leaves, then the arena of intermediates/adjoints for each
// program variant (0 = forward, 1 = forward + adjoint).
struct NetLayout {
  std::vector<int64_t> coff, poff;
  int64_t n_const = 0, leaf_region = 0, ptens_elems = 0;
  std::vector<int64_t> off[2];
  int64_t arena[2] = {0, 0};
};

static NetLayout make_layout(const Net &net) {
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

// Program arrays shared by the fused executor (LDS offsets) and the level
// executor (global arena offsets).
struct HostProgram {
  std::vector<DNet> nets_fwd, nets_grad;  // fused: one entry per batch network (level ones empty)
  std::vector<DOp> ops;
  std::vector<int32_t> tabs;
  std::vector<int32_t> recs;   // fused lane records, 4 ints x 64 lanes per op
  std::vector<double> consts;  // interleaved, converted to the dtype at upload
  std::vector<DParam> ptens;
  // distinct parametric tensors of the whole batch (bound once per parameter vector)
  std::vector<DParam> slots;
  std::map<std::tuple<int, int, double, int>, int> slot_of;
  int per_set = 0;
  int max_mem_fwd = 0, max_mem_grad = 0, max_comp = 0, max_ptens_elems = 0;
  int64_t max_mem_g[2] = {0, 0};  // global-arena programs: memory (elements), forward / adjoint
  std::map<std::string, int> program_of;  // fused program signature -> first network using it
  int n_programs = 0;
  bool generic[2] = {false, false};  // some op of a forward / adjoint program has no lane record
  // set-packed records for 4 and 2 sets per wave (index 0, 1): 4 ints x
  // W lanes per op; sets_ok: every op of every program has one
  std::vector<int32_t> srecs[2];
  bool sets_ok[2] = {true, true};
};

struct LevelNet {
  int net = 0;
  int n_comp = 0;
  int op_begin[2] = {0, 0}, n_ops[2] = {0, 0};  // into HostProgram::ops
  int64_t stride[2] = {0, 0};                   // elements per parameter vector
  int const_begin = 0, n_const = 0;             // into HostProgram::consts (elements)
  int ptens_begin = 0, n_ptens = 0;             // into HostProgram::ptens (absolute offsets)
  int64_t gbar_begin = 0, ptens_elems = 0;      // adjoint accumulators (variant 1)
  int chunk = 1;                                // parameter vectors per pass
  bool grad_ok = true;                          // the adjoint arena is addressable (< 2^31 elements)
};

// Level networks whose parameter vectors all fit in the arena at once run
// in bins: each network of a bin owns an arena region (and a region of
// component scalars), and step k of every network of the bin is one grouped
// launch per kind (thin contractions, leaf adjoints, matrix-core products
// per kernel variant). Rank-0 and seed steps keep launches of their own.
struct LevelBin {
  int lane = 0;                // stream lane (bins of different lanes run concurrently)
  int64_t part_off = 0;        // offset of its rank-0 partial sums (doubles)
  std::vector<int> lv;         // indices into tn_batch::level
  std::vector<int64_t> abase;  // arena region start (elements)
  std::vector<int64_t> sbase;  // component-scalar region start (doubles)
  // Matrix-core items of one kernel variant in a step.
  struct MGroup {
    int variant = 0, i0 = 0, n = 0, blocks = 0;
  };
  // per step: thin-contraction and leaf-adjoint items [t0, t0+nt) on tb
  // workgroups (into the variant's item array), matrix-core groups [g0,
  // g0+ng) of `mg`, the partial-tile sums of its split matrix-core items
  // [r0, r0+nr) on rb workgroups, separately launched ops [o0, o0+no) of
  // `other`
  struct Step {
    int t0 = 0, nt = 0, tb = 0, g0 = 0, ng = 0, r0 = 0, nr = 0, rb = 0, o0 = 0, no = 0;
  };
  std::vector<Step> steps[2];
  std::vector<MGroup> mg[2];
  std::vector<int> other[2];  // members whose op of the step runs on its own
};

// Most workgroups one item of a grouped launch takes.
static constexpr int64_t kGroupItemBlocks = 65536;

// Split summed index of matrix-core items: an item whose tiles over all
// parameter vectors number fewer than kSplitTarget workgroups (default;
// QTN_SPLIT_TARGET) is split into
// up to 64 ranges (at least 512 summed entries each) until it has about
// kSplitTarget; the partial tiles of one step and stream lane take at most
// kSplitStepBytes of scratch.
static constexpr int64_t kSplitTarget = 1024;
static constexpr int64_t kSplitStepBytes = int64_t(512) << 20;

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
static void out_offsets(const HostProgram &loc, const DOp &op, uint32_t c, int32_t &ox, int32_t &oy) {
  const uint32_t rest = c >> op.nFY;
  ox = op.x + (int32_t)host_pdep(rest >> op.nB, op.maskX);
  oy = op.y + (int32_t)host_pdep(c & ((1u << op.nFY) - 1u), op.maskY);
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    ox += loc.tabs[op.tabB + 2 * b];
    oy += loc.tabs[op.tabB + 2 * b + 1];
  }
}

// Lane records (see kRecLanes) of ops [first, first + n) of `loc`;
// `pt` are the network's parametric tensors (for leaf-gradient ops).
static void build_records(const HostProgram &loc, const std::vector<DParam> &pt, int first, int n,
                          std::vector<int32_t> &recs) {
  auto pack = [](int32_t a, int32_t b) { return (a & 0xffff) | (b << 16); };
  for (int o = first; o < first + n; ++o) {
    const DOp &op = loc.ops[o];
    const int lgOut = op.nFX + op.nB + op.nFY;
    // LDS offsets of output c's X and Y rows
    auto offs = [&](uint32_t c, int32_t &ox, int32_t &oy) { out_offsets(loc, op, c, ox, oy); };
    // (X, Y) offsets of summed entry k (tables of at most 2^12 entries)
    auto tab = [&](int k, int32_t &tx, int32_t &ty) {
      tx = loc.tabs[op.tab + 2 * k];
      ty = loc.tabs[op.tab + 2 * k + 1];
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
          if (l + (q << 6) < (1 << op.nFX)) a1 |= (loc.tabs[op.tab + l + (q << 6)] & 0xff) << (8 * q);
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
  }
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
    auto offs = [&](uint32_t c, int32_t &ox, int32_t &oy) { out_offsets(loc, op, c, ox, oy); };
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
    d.goff = (int32_t)(ln.gbar_begin + lay.poff[t] - lay.n_const);
    d.coeff = pt.coeff;
    d.slot = slot_for(hp, pt);
    hp.ptens.push_back(d);
  }
  for (int variant = 0; variant < 2; ++variant) {
    ln.op_begin[variant] = (int)hp.ops.size();
    ln.n_ops[variant] = variant == 0 ? p.n_fwd_ops : (int)p.ops.size();
    emit_ops(
        p, ln.n_ops[variant], hp, [&](int v) { return (int32_t)abs_off(net, lay, variant, v); },
        [&](const Op &op, DOp &d) {
          d.y = (int32_t)(ln.gbar_begin + lay.poff[op.aux0] - lay.n_const);
          d.aux0 = ln.ptens_begin + op.aux0;
          d.aux1 = op.aux1;
        });
  }
  // element offsets inside a set's arena are 32-bit: an adjoint arena past
  // 2^31 elements leaves the network usable for forward passes only
  ln.grad_ok = ln.stride[1] < kMaxArenaElems;
  int64_t per = ln.stride[ln.grad_ok ? 1 : 0] * eb;
  ln.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(max_sets, budget_bytes / std::max<int64_t>(1, per)));
  return ln;
}

template <typename T>
static hipError_t dalloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void **)p, n * sizeof(T));
}

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int with_grad = -1, n_sets = -1;
  const void *params = nullptr, *out = nullptr, *obj = nullptr, *grad = nullptr, *grad_net = nullptr;
  hipStream_t stream = nullptr;
  void clear() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

}  // namespace qtn

struct tn_batch {
  int dtype = 0, n_nets = 0, n_params = 0, max_sets = 0, block = 128;
  int spw[2] = {1, 1};                 // angle sets per wave of the fused executor (1, 2 or 4), forward / adjoint
  int64_t fused_budget = 0;            // LDS bytes a fused workgroup may use
  double offset = 0;
  std::vector<double> coef;
  qtn::HostProgram hp;
  std::vector<int32_t> task_net;       // fused networks, in cost order
  std::vector<int32_t> gtask_net;      // networks on the global-arena fused executor, in cost order
  struct GLayout { int lds = 0, grid = 0, scratch_off = 0, scal_off = 0, gacc_off = 0, red_off = 0; } gl[2];
  int64_t gstride = 0;                 // elements per global-arena slot
  int gslots = 0;                      // slots (= most workgroups of one launch)
  std::vector<qtn::LevelNet> level;    // networks on the level executor
  std::vector<qtn::LevelBin> lbins;    // level networks run with grouped launches
  std::vector<int> lsolo;              // level networks run one by one, in chunks of parameter vectors
  qtn::LItem *d_litems[2] = {nullptr, nullptr};
  int32_t *d_lblk[2] = {nullptr, nullptr};  // the items' first-workgroup indices (compact copy)
  size_t litem_cap[2] = {0, 0};
  void *d_lsplit = nullptr;                       // partial tiles of split matrix-core items
  size_t lsplit_cap = 0;                          // its bytes
  int64_t lsplit_off[2][2] = {{0, 0}, {0, 0}};    // [program variant][lane]: region start (elements)
  int64_t split_target = 0;                       // workgroups a split item aims at (0: no splits)
  // device
  qtn::DNet *d_nets_fwd = nullptr, *d_nets_grad = nullptr;
  qtn::DOp *d_ops = nullptr;
  int4 *d_recs = nullptr, *d_srecs[2] = {nullptr, nullptr};
  int32_t *d_tabs = nullptr, *d_task_net = nullptr, *d_gtask_net = nullptr;
  void *d_garena = nullptr;            // global-arena slots
  void *d_consts = nullptr;
  qtn::DParam *d_ptens = nullptr, *d_slots = nullptr;
  void *d_bound = nullptr, *d_dbound = nullptr;
  double *d_val = nullptr, *d_gnet = nullptr, *d_coef = nullptr;
  void *d_larena = nullptr;            // level executor arena
  double *d_lscal = nullptr;           // level executor component scalars
  double *d_lpart = nullptr;           // level executor partial sums
  int lds_fwd = 0, lds_grad = 0, grid_fwd = 0, grid_grad = 0;
  int scratch_off[2], scal_off[2], gacc_off[2], red_off[2], gbar_off[2], set_stride[2];
  double flops_fwd = 0, bytes_fwd = 0, flops_grad = 0, bytes_grad = 0;
  int64_t level_bytes = 0;
  std::map<std::string, int> use_mfma;  // autotuner: shape class of a large op -> 1 MFMA, 0 thin
  int mfma_prec = TN_MFMA_FP32;          // matrix-core precision of large steps (complex128: TN_MFMA_FP64)
  bool poisoned = false;
  qtn::GraphCache gc;
  // kernel timing (tn_batch_kernel_timing): event pairs around fused launches
  bool timing = false, capturing = false;
  // with work on two or more executors (or two level lanes), the
  // global-arena executor runs on side[0] and the level lanes on side[1] and
  // side[2], forked from the caller's stream after binding and joined before
  // the combine, so the executors (independent networks) overlap
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
};

namespace qtn {

static int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return TN_EDEVICE;
}

#define HIPCHK(call)                                    \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hip_fail(_e, #call);   \
  } while (0)

static void drop_timing_events(tn_batch *b) {
  for (auto &pr : b->tev) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  b->tev.clear();
}

static void free_batch_dev(tn_batch *b) {
  b->gc.clear();
  drop_timing_events(b);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  b->ev_fork = nullptr;
  for (int i = 0; i < 3; ++i) {
    if (b->ev_join[i]) (void)hipEventDestroy(b->ev_join[i]);
    if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    b->ev_join[i] = nullptr;
    b->side[i] = nullptr;
  }
  void *ptrs[] = {b->d_nets_fwd, b->d_nets_grad, b->d_ops, b->d_recs, b->d_srecs[0], b->d_srecs[1], b->d_tabs, b->d_task_net, b->d_gtask_net, b->d_garena, b->d_consts, b->d_ptens,
                  b->d_slots, b->d_bound, b->d_dbound, b->d_val, b->d_gnet, b->d_coef, b->d_larena, b->d_lscal,
                  b->d_lpart, b->d_litems[0], b->d_litems[1], b->d_lblk[0], b->d_lblk[1], b->d_lsplit};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
}

static std::string shape_class(int dtype, const DOp &op, int prec);

// Matrix-core precision a level op runs with (0: a thin kernel).
static int level_prec(const tn_batch *b, const DOp &op) {
  if (!mfma_eligible(b->dtype, op)) return 0;
  auto it = b->use_mfma.find(shape_class(b->dtype, op, b->mfma_prec));
  return it == b->use_mfma.end() || it->second ? b->mfma_prec : 0;
}

// Item lists of the level bins for the current matrix-core choices,
// uploaded to the device. Runs after every change of those choices, never
// under capture.
static int build_level_items(tn_batch *b) {
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  int64_t split_need[2][2] = {{0, 0}, {0, 0}};  // [variant][lane]: scratch elements
  for (int v = 0; v < 2; ++v) {
    std::vector<LItem> items;
    for (LevelBin &bn : b->lbins) {
      bn.steps[v].clear();
      bn.other[v].clear();
      bn.mg[v].clear();
      int n_steps = 0;
      for (int l : bn.lv) n_steps = std::max(n_steps, b->level[l].n_ops[v]);
      for (int k = 0; k < n_steps; ++k) {
        LevelBin::Step stp;
        {
          // thin contractions and leaf adjoints: one launch
          const int first = (int)items.size();
          int blocks = 0;
          for (size_t j = 0; j < bn.lv.size(); ++j) {
            const LevelNet &ln = b->level[bn.lv[j]];
            if (k >= ln.n_ops[v]) continue;
            const DOp &op = b->hp.ops[ln.op_begin[v] + k];
            const bool thin = op.type == OP_CONTRACT && level_prec(b, op) == 0;
            const bool leaf = op.type == OP_LEAFGRAD;
            if (!(thin || leaf)) continue;
            const int lg = thin ? op.nFX + op.nB + op.nFY : op.nFX;
            int64_t work = ((int64_t)1 << lg) * b->max_sets;
            LItem it{};
            if (thin) {
              // lanes per output: at least 8 summed entries each, up to 64,
              // while the step has fewer than 2^20 (output, lane) pairs
              int lgs = 0;
              while ((int64_t(1) << lgs) < b->max_sets) ++lgs;
              it.lgl = std::max(0, std::min({6, op.nS - 3, 20 - lg - lgs}));
              work <<= it.lgl;
              // many outputs: four per lane instead (shared X reads)
              if (it.lgl == 0 && lg + lgs >= 16 && (op.nFY >= 2 || (op.nFY == 0 && op.nB == 0 && op.nFX >= 8))) {
                // 64 apart along Y (>= 8 Y-only bits) or X (X-only output bits), else consecutive
                it.lgl = op.nFY >= 8 ? -2 : op.nFY == 0 ? -3 : -1;
                work >>= 2;
              }
            }
            it.op = op;
            pack_runs(op.maskX, it.ru.runsX);
            pack_runs(op.maskY, it.ru.runsY);
            it.base = bn.abase[j];
            it.stride = ln.stride[v];
            it.blk0 = blocks;
            blocks += (int)std::max<int64_t>(1, std::min<int64_t>(kGroupItemBlocks, (work + 255) / 256));
            items.push_back(it);
          }
          stp.t0 = first;
          stp.nt = (int)items.size() - first;
          stp.tb = blocks;
        }
        // matrix-core products, grouped by kernel variant
        std::vector<std::pair<int, int>> mf;  // (variant, member)
        stp.o0 = (int)bn.other[v].size();
        for (size_t j = 0; j < bn.lv.size(); ++j) {
          const LevelNet &ln = b->level[bn.lv[j]];
          if (k >= ln.n_ops[v]) continue;
          const DOp &op = b->hp.ops[ln.op_begin[v] + k];
          if (op.type == OP_LEAFGRAD) continue;
          if (op.type == OP_CONTRACT) {
            const int prec = level_prec(b, op);
            if (prec) mf.emplace_back(mfma_variant(op, prec), (int)j);
            continue;
          }
          bn.other[v].push_back((int)j);
        }
        stp.no = (int)bn.other[v].size() - stp.o0;
        std::stable_sort(mf.begin(), mf.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
          return x.first < y.first;
        });
        stp.g0 = (int)bn.mg[v].size();
        std::vector<LItem> splits;
        int64_t zoff = 0;  // scratch elements of this step's split items
        for (size_t q = 0; q < mf.size(); ++q) {
          if (q == 0 || mf[q].first != mf[q - 1].first) {
            LevelBin::MGroup g;
            g.variant = mf[q].first;
            g.i0 = (int)items.size();
            bn.mg[v].push_back(g);
          }
          LevelBin::MGroup &g = bn.mg[v].back();
          const int j = mf[q].second;
          const LevelNet &ln = b->level[bn.lv[j]];
          LItem it{};
          it.op = b->hp.ops[ln.op_begin[v] + k];
          pack_runs(it.op.maskX, it.ru.runsX);
          pack_runs(it.op.maskY, it.ru.runsY);
          it.base = bn.abase[j];
          it.stride = ln.stride[v];
          it.blk0 = g.blocks;
          const int64_t wg = (int64_t)mfma_tiles(it.op) * b->max_sets;
          const int64_t part = ((int64_t)b->max_sets << (it.op.nFX + it.op.nFY));  // elements per range
          int ls = 0;
          while (ls < 6 && it.op.nS - ls > 9 && (wg << ls) < b->split_target &&
                 (zoff + (part << (ls + 1))) * eb <= kSplitStepBytes)
            ++ls;
          if (ls > 0) {
            it.lgl = ls;
            it.zs = zoff;
            zoff += part << ls;
            splits.push_back(it);
          }
          g.blocks += (int)(wg << ls);
          ++g.n;
          items.push_back(it);
        }
        stp.ng = (int)bn.mg[v].size() - stp.g0;
        // sums of the split items' partial tiles
        stp.r0 = (int)items.size();
        stp.nr = (int)splits.size();
        for (LItem &it : splits) {
          it.blk0 = stp.rb;
          const int64_t outs = (int64_t)b->max_sets << (it.op.nFX + it.op.nFY);
          stp.rb += (int)std::max<int64_t>(1, std::min<int64_t>(kGroupItemBlocks, (outs + 255) / 256));
          items.push_back(it);
        }
        split_need[v][bn.lane] = std::max(split_need[v][bn.lane], zoff);
        bn.steps[v].push_back(stp);
      }
    }
    if (items.empty()) continue;
    if (items.size() > b->litem_cap[v]) {
      // earlier launches may still read the old lists
      HIPCHK(hipDeviceSynchronize());
      if (b->d_litems[v]) HIPCHK(hipFree(b->d_litems[v]));
      if (b->d_lblk[v]) HIPCHK(hipFree(b->d_lblk[v]));
      b->d_litems[v] = nullptr;
      b->d_lblk[v] = nullptr;
      b->litem_cap[v] = 0;
      HIPCHK(hipMalloc((void **)&b->d_litems[v], items.size() * sizeof(LItem)));
      HIPCHK(hipMalloc((void **)&b->d_lblk[v], items.size() * sizeof(int32_t)));
      b->litem_cap[v] = items.size();
    }
    std::vector<int32_t> blk(items.size());
    for (size_t i = 0; i < items.size(); ++i) blk[i] = items[i].blk0;
    // earlier launches may still read the old lists
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(b->d_litems[v], items.data(), items.size() * sizeof(LItem), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_lblk[v], blk.data(), blk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  // split scratch: lane 0's region, then lane 1's (the lanes run concurrently)
  size_t need = 0;
  for (int v = 0; v < 2; ++v) {
    b->lsplit_off[v][0] = 0;
    b->lsplit_off[v][1] = split_need[v][0];
    need = std::max(need, (size_t)(split_need[v][0] + split_need[v][1]) * eb);
  }
  if (need > b->lsplit_cap) {
    HIPCHK(hipDeviceSynchronize());
    if (b->d_lsplit) HIPCHK(hipFree(b->d_lsplit));
    b->d_lsplit = nullptr;
    b->lsplit_cap = 0;
    HIPCHK(hipMalloc(&b->d_lsplit, need));
    b->lsplit_cap = need;
  }
  b->gc.clear();
  return TN_OK;
}

// 64-lane workgroups whose programs have a lane record for every op run a
// kernel instance without the descriptor path (fewer registers live across
// the op loop).
static bool rec_only(const tn_batch *b, int variant) { return b->block == kRecLanes && !b->hp.generic[variant]; }

// LDS bytes of the set-packed layout with S sets per wave: per set its
// memory, component scalars and gradient sums. The sets' regions start 64
// bytes apart modulo the 256-byte bank cycle, so the same lane of different
// sets reads different banks.
static int set_lds_layout(const tn_batch *b, int S, int variant, int *stride, int *scal_off, int *gacc_off) {
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
static bool sets_fit(const tn_batch *b, int S, int64_t budget, int variant) {
  if (b->task_net.empty() || !b->hp.sets_ok[S == 4 ? 0 : 1]) return false;
  int st, so, go;
  return set_lds_layout(b, S, variant, &st, &so, &go) <= std::min<int64_t>(budget, 64 * 1024);
}

static int layout_lds(tn_batch *b, int variant) {
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const int mem = variant == 0 ? b->hp.max_mem_fwd : b->hp.max_mem_grad;
  auto al = [](int x) { return (x + 15) & ~15; };
  int dev = 0, cus = 0, per_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (b->spw[variant] > 1) {
    const int o = set_lds_layout(b, b->spw[variant], variant, &b->set_stride[variant], &b->scal_off[variant], &b->gacc_off[variant]);
    b->scratch_off[variant] = b->red_off[variant] = b->gbar_off[variant] = 0;
    if (o > kLdsCap) {
      set_error("fused executor: LDS layout of " + std::to_string(o) + " bytes exceeds 160 KiB");
      return TN_ENOMEM;
    }
    (variant == 0 ? b->lds_fwd : b->lds_grad) = o;
    const void *k = fused_sets_kernel_ptr(b->dtype, variant == 1, b->spw[variant]);
    if (o > 64 * 1024) HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, o));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64, o));
    (variant == 0 ? b->grid_fwd : b->grid_grad) = std::max(1, per_cu) * std::max(1, cus);
    return TN_OK;
  }
  b->set_stride[variant] = 0;
  int o = al(mem * eb);
  b->scratch_off[variant] = o;
  o = al(o + b->block * eb);
  b->scal_off[variant] = o;
  o = al(o + std::max(1, b->hp.max_comp) * 16);
  b->gacc_off[variant] = o;
  o = al(o + std::max(1, b->n_params) * 8);
  b->red_off[variant] = o;
  o = al(o + 16 * 8);
  b->gbar_off[variant] = o;
  if (o > kLdsCap) {
    set_error("fused executor: LDS layout of " + std::to_string(o) + " bytes exceeds 160 KiB");
    return TN_ENOMEM;
  }
  (variant == 0 ? b->lds_fwd : b->lds_grad) = o;
  const void *k = fused_kernel_ptr(b->dtype, b->block, variant == 1, rec_only(b, variant), false);
  if (o > 64 * 1024) HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, o));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, b->block, o));
  int grid = std::max(1, per_cu) * std::max(1, cus);
  (variant == 0 ? b->grid_fwd : b->grid_grad) = grid;
  return TN_OK;
}

// Global-arena fused executor: LDS holds only the scratch, the component
// scalars, the gradient sums and the reduction slots; the arena has one slot
// of `gstride` elements per workgroup.
static int layout_gmem(tn_batch *b) {
  if (b->gtask_net.empty()) return TN_OK;
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  auto al = [](int x) { return (x + 15) & ~15; };
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int grid_max = 0;
  for (int v = 0; v < 2; ++v) {
    tn_batch::GLayout &g = b->gl[v];
    g.scratch_off = 0;
    int o = al(256 * eb);
    g.scal_off = o;
    o = al(o + std::max(1, b->hp.max_comp) * 16);
    g.gacc_off = o;
    o = al(o + std::max(1, b->n_params) * 8);
    g.red_off = o;
    o = al(o + 16 * 8);
    g.lds = o;
    int per_cu = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel_ptr(b->dtype, 256, v == 1, false, true), 256, o));
    g.grid = std::max(1, per_cu) * std::max(1, cus);
    grid_max = std::max(grid_max, g.grid);
  }
  b->gstride = (std::max(b->hp.max_mem_g[0], b->hp.max_mem_g[1]) + 63) & ~int64_t(63);
  b->gslots = (int)std::max<int64_t>(1, std::min<int64_t>(grid_max, kGmemBudget / (b->gstride * eb)));
  return TN_OK;
}

int batch_create(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch **out) {
  if (!nets || n_nets < 1 || max_sets < 1 || !out) {
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
  std::unique_ptr<tn_batch> b(new tn_batch());
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
  if (const char *env = std::getenv("QTN_FUSED_LDS_MAX")) fused_max = std::atoll(env);
  int64_t gmem_max = kGmemMaxMacs;  // QTN_GMEM_MAX_MACS=0 turns the global-arena executor off
  if (const char *env = std::getenv("QTN_GMEM_MAX_MACS")) gmem_max = std::atoll(env);
  int64_t level_budget = kLevelBudget;  // QTN_LEVEL_BUDGET (bytes): level arena limit
  if (const char *env = std::getenv("QTN_LEVEL_BUDGET")) level_budget = std::max<int64_t>(1, std::atoll(env));
  b->split_target = kSplitTarget;  // QTN_SPLIT_TARGET=0 keeps every matrix-core sum on one workgroup
  if (const char *env = std::getenv("QTN_SPLIT_TARGET")) b->split_target = std::max<int64_t>(0, std::atoll(env));
  std::vector<double> cost(n_nets);
  std::vector<int> fused_ids, gmem_ids;
  int maxbits = 0;
  for (int i = 0; i < n_nets; ++i) {
    const Net *n = reinterpret_cast<const Net *>(nets[i]);
    NetLayout lay = make_layout(*n);
    cost[i] = n->gplan.flops + n->gplan.flops_grad + 1e3 * n->gplan.ops.size();
    b->flops_fwd += n->gplan.flops;
    b->bytes_fwd += n->gplan.bytes;
    b->flops_grad += n->gplan.flops_grad;
    b->bytes_grad += n->gplan.bytes_grad;
    double max_macs = 0, tot_macs = 0;
    for (const Op &op : n->gplan.ops)
      if (op.type == OP_CONTRACT || op.type == OP_SCALAR) {
        const double m = std::ldexp(1.0, op.nFX + op.nB + op.nS + op.nFY);
        max_macs = std::max(max_macs, m);
        tot_macs += m;
      }
    const int64_t mem_elems = lay.leaf_region + std::max(lay.arena[0], lay.arena[1]);
    if (fused_lds_need(*n, lay, eb, b->n_params) <= fused_max) {
      append_fused(*n, lay, b->hp, false);
      fused_ids.push_back(i);
      maxbits = std::max(maxbits, n->gplan.peak_bits);
    } else if (tot_macs <= (double)gmem_max && max_macs <= (double)gmem_max / 16 && mem_elems < kMaxArenaElems &&
               mem_elems * eb <= kGmemBudget / 256) {
      append_fused(*n, lay, b->hp, true);
      gmem_ids.push_back(i);
    } else {
      b->hp.nets_fwd.push_back(DNet{});
      b->hp.nets_grad.push_back(DNet{});
      b->level.push_back(append_level(*n, lay, b->hp, i, eb, level_budget, max_sets));
      if (b->level.back().stride[0] >= kMaxArenaElems) {
        set_error("tn_batch_create: network " + std::to_string(i) + " needs " + std::to_string(b->level.back().stride[0]) +
                  " elements of working memory per parameter vector; the executor addresses at most 2^31");
        return TN_ENOMEM;
      }
    }
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
  int rc;
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
    if (want[v] == 4 && sets_fit(b.get(), 4, fused_max, v)) b->spw[v] = 4;
    else if (want[v] >= 2 && sets_fit(b.get(), 2, fused_max, v)) b->spw[v] = 2;
  }
  if ((rc = layout_lds(b.get(), 0)) != TN_OK) return rc;
  if ((rc = layout_lds(b.get(), 1)) != TN_OK) return rc;
  if ((rc = layout_gmem(b.get())) != TN_OK) return rc;

  tn_batch *B = b.get();
  auto fail = [&](hipError_t e, const char *w) {
    free_batch_dev(B);
    return hip_fail(e, w);
  };
  hipError_t e;
  const HostProgram &hp = b->hp;
  if ((e = dalloc(&b->d_nets_fwd, hp.nets_fwd.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_nets_grad, hp.nets_grad.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_ops, hp.ops.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_tabs, hp.tabs.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_recs, hp.recs.size() / 4)) != hipSuccess) return fail(e, "hipMalloc");
  for (int i = 0; i < 2; ++i)
    if ((e = dalloc(&b->d_srecs[i], hp.srecs[i].size() / 4)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_task_net, b->task_net.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_gtask_net, b->gtask_net.size())) != hipSuccess) return fail(e, "hipMalloc");
  if (!b->gtask_net.empty() &&
      (e = dalloc((char **)&b->d_garena, (size_t)b->gslots * b->gstride * eb)) != hipSuccess)
    return fail(e, "hipMalloc (global arena)");
  if ((e = dalloc((char **)&b->d_consts, hp.consts.size() / 2 * eb)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_ptens, hp.ptens.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_slots, hp.slots.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc((char **)&b->d_bound, (size_t)max_sets * std::max(1, hp.per_set) * eb)) != hipSuccess)
    return fail(e, "hipMalloc");
  if ((e = dalloc((char **)&b->d_dbound, (size_t)max_sets * std::max(1, hp.per_set) * eb)) != hipSuccess)
    return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_val, (size_t)n_nets * max_sets * 2)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_gnet, (size_t)n_nets * max_sets * std::max(1, b->n_params))) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_coef, (size_t)n_nets)) != hipSuccess) return fail(e, "hipMalloc");
  {
    // bins: level networks that take every parameter vector at once, packed
    // in order while their regions fit the level budget together
    int64_t arena = 0, scal = 0, part = 0, bin_elems = 0, bin_scal = 0;
    for (int l = 0; l < (int)b->level.size(); ++l) {
      const LevelNet &ln = b->level[l];
      const int64_t per = ln.stride[ln.grad_ok ? 1 : 0];
      part = std::max(part, (int64_t)ln.chunk * kScalarParts * 2);
      if (ln.chunk < max_sets) {
        b->lsolo.push_back(l);
        arena = std::max(arena, per * ln.chunk * eb);
        scal = std::max(scal, (int64_t)ln.chunk * std::max(1, ln.n_comp) * 2);
        continue;
      }
      const int64_t need = (per * max_sets + 63) / 64 * 64;
      if (b->lbins.empty() || (bin_elems + need) * eb > level_budget) {
        b->lbins.emplace_back();
        bin_elems = bin_scal = 0;
      }
      LevelBin &bn = b->lbins.back();
      bn.lv.push_back(l);
      bn.abase.push_back(bin_elems);
      bn.sbase.push_back(bin_scal);
      bin_elems += need;
      bin_scal += (int64_t)max_sets * std::max(1, ln.n_comp) * 2;
      arena = std::max(arena, bin_elems * eb);
      scal = std::max(scal, bin_scal);
    }
    // one group of several networks: split it into two halves that run
    // concurrently on two streams (regions stay disjoint: the halves take
    // consecutive ranges of the same arena), networks dealt alternately
    if (b->lbins.size() == 1 && b->lbins[0].lv.size() >= 2 && b->lsolo.empty()) {
      const LevelBin one = b->lbins[0];
      b->lbins.assign(2, LevelBin{});
      int64_t off = 0, soff = 0;
      for (int h = 0; h < 2; ++h) {
        LevelBin &bn = b->lbins[h];
        bn.lane = h;
        bn.part_off = h * part;
        for (size_t j = h; j < one.lv.size(); j += 2) {
          const LevelNet &ln = b->level[one.lv[j]];
          bn.lv.push_back(one.lv[j]);
          bn.abase.push_back(off);
          bn.sbase.push_back(soff);
          off += (ln.stride[ln.grad_ok ? 1 : 0] * max_sets + 63) / 64 * 64;
          soff += (int64_t)max_sets * std::max(1, ln.n_comp) * 2;
        }
      }
      part *= 2;
    }
    b->level_bytes = arena;
    if (!b->level.empty()) {
      if ((e = dalloc((char **)&b->d_larena, (size_t)arena)) != hipSuccess) return fail(e, "hipMalloc (level arena)");
      if ((e = dalloc(&b->d_lscal, (size_t)scal)) != hipSuccess) return fail(e, "hipMalloc");
      if ((e = dalloc(&b->d_lpart, (size_t)part)) != hipSuccess) return fail(e, "hipMalloc");
    }
  }
  // side streams only for the executors that have work (streams share the
  // few hardware queues: an idle stream could take a busy one's queue)
  const bool two_lanes = b->lbins.size() == 2 && b->lbins[1].lane == 1;
  if ((!b->task_net.empty()) + (!b->gtask_net.empty()) + (!b->level.empty()) >= 2 || two_lanes) {
    if ((e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming)) != hipSuccess) return fail(e, "hipEventCreate");
    const bool need[3] = {!b->gtask_net.empty(), !b->level.empty(), two_lanes};
    for (int i = 0; i < 3; ++i) {
      if (!need[i]) continue;
      if ((e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking)) != hipSuccess) return fail(e, "hipStreamCreate");
      if ((e = hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming)) != hipSuccess) return fail(e, "hipEventCreate");
    }
  }
  std::vector<float> cf;
  const void *csrc = hp.consts.data();
  if (b->dtype == TN_C64) {
    cf.assign(hp.consts.begin(), hp.consts.end());
    csrc = cf.data();
  }
  struct Up { void *d; const void *h; size_t n; } ups[] = {
      {b->d_nets_fwd, hp.nets_fwd.data(), hp.nets_fwd.size() * sizeof(DNet)},
      {b->d_nets_grad, hp.nets_grad.data(), hp.nets_grad.size() * sizeof(DNet)},
      {b->d_ops, hp.ops.data(), hp.ops.size() * sizeof(DOp)},
      {b->d_tabs, hp.tabs.data(), hp.tabs.size() * sizeof(int32_t)},
      {b->d_recs, hp.recs.data(), hp.recs.size() * sizeof(int32_t)},
      {b->d_srecs[0], hp.srecs[0].data(), hp.srecs[0].size() * sizeof(int32_t)},
      {b->d_srecs[1], hp.srecs[1].data(), hp.srecs[1].size() * sizeof(int32_t)},
      {b->d_task_net, b->task_net.data(), b->task_net.size() * sizeof(int32_t)},
      {b->d_gtask_net, b->gtask_net.data(), b->gtask_net.size() * sizeof(int32_t)},
      {b->d_consts, csrc, hp.consts.size() / 2 * eb},
      {b->d_ptens, hp.ptens.data(), hp.ptens.size() * sizeof(DParam)},
      {b->d_slots, hp.slots.data(), hp.slots.size() * sizeof(DParam)},
      {b->d_coef, b->coef.data(), b->coef.size() * sizeof(double)},
  };
  for (auto &u : ups)
    if (u.n && (e = hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "hipMemcpy");
  if ((rc = build_level_items(B)) != TN_OK) {
    free_batch_dev(B);
    return rc;
  }
  *out = b.release();
  return TN_OK;
}

// Key of a large op for the autotuner: dtype, free/summed bit counts and
// which operands are read with the summed index contiguous.
static std::string shape_class(int dtype, const DOp &op, int prec) {
  return std::to_string(dtype) + "p" + std::to_string(prec) + ":" + std::to_string(op.nFX) + "," + std::to_string(op.nS) + "," +
         std::to_string(op.nFY) + ":" + std::to_string(!(op.maskX & 1u)) + std::to_string(!(op.maskY & 1u));
}

static int run_batch(tn_batch *b, bool grad, const double *params, int n_sets, double *out, double *obj, double *gobj,
                     double *gnet_out, hipStream_t st) {
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  if ((!params && b->n_params > 0) || n_sets < 1 || n_sets > b->max_sets) {
    set_error("batch run: n_sets out of range or params NULL");
    return TN_EINVAL;
  }
  if (grad)
    for (const LevelNet &ln : b->level)
      if (!ln.grad_ok) {
        set_error("batch gradient: network " + std::to_string(ln.net) +
                  " needs more than 2^31 elements of adjoint working memory per parameter vector");
        return TN_ENOMEM;
      }
  const int v = grad ? 1 : 0;
  FusedArgs a{};
  a.nets = grad ? b->d_nets_grad : b->d_nets_fwd;
  a.ops = b->d_ops;
  a.recs = b->d_recs;
  a.tabs = b->d_tabs;
  a.consts = b->d_consts;
  a.ptens = b->d_ptens;
  a.bound = b->d_bound;
  a.dbound = b->d_dbound;
  a.per_set = b->hp.per_set;
  a.task_net = b->d_task_net;
  // network-major output; the internal buffer is used when the caller's
  // layout would not match or no pointer is given
  a.out_val = out ? out : b->d_val;
  a.out_grad = gnet_out ? gnet_out : b->d_gnet;
  a.n_params = b->n_params;
  a.n_sets = n_sets;
  a.n_tasks = (int)b->task_net.size() * n_sets;
  a.scratch_off = b->scratch_off[v];
  a.scal_off = b->scal_off[v];
  a.gacc_off = b->gacc_off[v];
  a.red_off = b->red_off[v];
  a.gbar_off = b->gbar_off[v];
  hipError_t e = launch_bind(b->dtype, b->d_slots, (int)b->hp.slots.size(), params, b->n_params, n_sets,
                             b->hp.per_set, b->d_bound, grad ? b->d_dbound : nullptr, st);
  if (e != hipSuccess) {
    b->poisoned = true;
    return hip_fail(e, "binding launch");
  }
  // streams of the global-arena (sg) and level (sl: lane 0, sl1: lane 1)
  // executors: forked when two or more of them have work
  hipStream_t sg = st, sl = st, sl1 = st;
  const bool fork = b->ev_fork != nullptr;
  if (fork) {
    e = hipEventRecord(b->ev_fork, st);
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
      if (b->side[i]) e = hipStreamWaitEvent(b->side[i], b->ev_fork, 0);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "stream fork");
    }
    if (b->side[0]) sg = b->side[0];
    if (b->side[1]) sl = sl1 = b->side[1];
    if (b->side[2]) sl1 = b->side[2];
  }
  const int spw = b->spw[v];
  if (spw > 1) {
    a.recs = b->d_srecs[spw == 4 ? 0 : 1];
    a.set_stride = b->set_stride[v];
    a.max_comp = std::max(1, b->hp.max_comp);
    a.n_groups = (n_sets + spw - 1) / spw;
    a.n_tasks = (int)b->task_net.size() * a.n_groups;
  }
  if (a.n_tasks > 0) {
    // resident workgroups, balanced so every one runs the same number of tasks
    const int cap = std::max(1, std::min(grad ? b->grid_grad : b->grid_fwd, a.n_tasks));
    const int rounds = (a.n_tasks + cap - 1) / cap;
    const int grid = (a.n_tasks + rounds - 1) / rounds;
    a.per_block = rounds;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (b->timing && !b->capturing && b->tev.size() < 4096 && hipEventCreate(&t0) == hipSuccess) {
      if (hipEventCreate(&t1) != hipSuccess || hipEventRecord(t0, st) != hipSuccess) {
        (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        t0 = t1 = nullptr;
      }
    }
    if (spw > 1)
      e = launch_fused_sets(b->dtype, grad, spw, a, grid, grad ? b->lds_grad : b->lds_fwd, st);
    else
      e = launch_fused(b->dtype, b->block, grad, rec_only(b, v), false, a, grid, grad ? b->lds_grad : b->lds_fwd, st);
    if (t0) {
      if (e == hipSuccess && hipEventRecord(t1, st) == hipSuccess) {
        b->tev.emplace_back(t0, t1);
      } else {
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
      }
    }
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "fused executor launch");
    }
  }
  if (!b->gtask_net.empty()) {
    const tn_batch::GLayout &gl = b->gl[v];
    FusedArgs g = a;
    g.recs = b->d_recs;
    g.task_net = b->d_gtask_net;
    g.n_tasks = (int)b->gtask_net.size() * n_sets;
    g.scratch_off = gl.scratch_off;
    g.scal_off = gl.scal_off;
    g.gacc_off = gl.gacc_off;
    g.red_off = gl.red_off;
    g.garena = b->d_garena;
    g.garena_stride = b->gstride;
    const int cap = std::max(1, std::min(std::min(gl.grid, b->gslots), g.n_tasks));
    const int rounds = (g.n_tasks + cap - 1) / cap;
    g.per_block = rounds;
    e = launch_fused(b->dtype, 256, grad, false, true, g, (g.n_tasks + rounds - 1) / rounds, gl.lds, sg);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "global-arena executor launch");
    }
  }
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  for (const LevelBin &bn : b->lbins) {
    hipStream_t bs = bn.lane == 1 ? sl1 : sl;
    auto args = [&](size_t j) {
      const LevelNet &ln = b->level[bn.lv[j]];
      LevelArgs la{};
      la.arena = (char *)b->d_larena + bn.abase[j] * eb;
      la.stride = ln.stride[v];
      la.n_sets = n_sets;
      la.scal = b->d_lscal + bn.sbase[j];
      la.n_comp = ln.n_comp;
      la.part = b->d_lpart + bn.part_off;
      return la;
    };
    for (size_t j = 0; j < bn.lv.size() && e == hipSuccess; ++j) {
      const LevelNet &ln = b->level[bn.lv[j]];
      e = level_setup(b->dtype, args(j), (const char *)b->d_consts + (size_t)ln.const_begin * eb, ln.n_const,
                      b->d_ptens + ln.ptens_begin, ln.n_ptens, b->d_bound, b->hp.per_set, 0, (int)ln.gbar_begin,
                      grad ? (int)ln.ptens_elems : 0, bs);
    }
    for (const LevelBin::Step &stp : bn.steps[v]) {
      if (e == hipSuccess)
        e = level_group(b->dtype, b->d_litems[v] + stp.t0, b->d_lblk[v] + stp.t0, stp.nt, stp.tb, b->d_larena, n_sets,
                        b->d_tabs, bs);
      void *split = b->d_lsplit ? (char *)b->d_lsplit + b->lsplit_off[v][bn.lane] * eb : nullptr;
      for (int g = stp.g0; g < stp.g0 + stp.ng && e == hipSuccess; ++g) {
        const LevelBin::MGroup &mg = bn.mg[v][g];
        e = mfma_group(mg.variant, b->d_litems[v] + mg.i0, b->d_lblk[v] + mg.i0, mg.n, mg.blocks, b->d_larena, split,
                       n_sets, b->d_tabs, bs);
      }
      if (e == hipSuccess && stp.nr > 0)
        e = mfma_split_reduce(b->dtype, b->d_litems[v] + stp.r0, b->d_lblk[v] + stp.r0, stp.nr, stp.rb, b->d_larena,
                              split, n_sets, bs);
      for (int q = stp.o0; q < stp.o0 + stp.no && e == hipSuccess; ++q) {
        const int j = bn.other[v][q];
        const LevelNet &ln = b->level[bn.lv[j]];
        const DOp &op = b->hp.ops[ln.op_begin[v] + (int)(&stp - bn.steps[v].data())];
        e = level_op(b->dtype, args(j), op, b->d_tabs, 0, bs);
      }
    }
    for (size_t j = 0; j < bn.lv.size() && e == hipSuccess; ++j) {
      const LevelNet &ln = b->level[bn.lv[j]];
      e = level_finish(b->dtype, args(j), b->d_ptens + ln.ptens_begin, ln.n_ptens, b->d_dbound, b->hp.per_set, 0, ln.net,
                       n_sets, b->n_params, a.out_val, a.out_grad, grad ? 1 : 0, bs);
    }
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "level executor launch");
    }
  }
  for (int l : b->lsolo) {
    const LevelNet &ln = b->level[l];
    for (int s0 = 0; s0 < n_sets; s0 += ln.chunk) {
      LevelArgs la{};
      la.arena = b->d_larena;
      la.stride = ln.stride[v];
      la.n_sets = std::min(ln.chunk, n_sets - s0);
      la.scal = b->d_lscal;
      la.n_comp = ln.n_comp;
      la.part = b->d_lpart;
      e = level_setup(b->dtype, la, (const char *)b->d_consts + (size_t)ln.const_begin * eb, ln.n_const,
                      b->d_ptens + ln.ptens_begin, ln.n_ptens, b->d_bound, b->hp.per_set, s0, (int)ln.gbar_begin,
                      grad ? (int)ln.ptens_elems : 0, sl);
      for (int o = 0; o < ln.n_ops[v] && e == hipSuccess; ++o) {
        const DOp &op = b->hp.ops[ln.op_begin[v] + o];
        e = level_op(b->dtype, la, op, b->d_tabs, level_prec(b, op), sl);
      }
      if (e == hipSuccess)
        e = level_finish(b->dtype, la, b->d_ptens + ln.ptens_begin, ln.n_ptens, b->d_dbound, b->hp.per_set, s0, ln.net,
                         n_sets, b->n_params, a.out_val, a.out_grad, grad ? 1 : 0, sl);
      if (e != hipSuccess) {
        b->poisoned = true;
        return hip_fail(e, "level executor launch");
      }
    }
  }
  if (fork) {
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
      if (!b->side[i]) continue;
      e = hipEventRecord(b->ev_join[i], b->side[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_join[i], 0);
    }
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "stream join");
    }
  }
  if (obj || (grad && gobj)) {
    e = launch_combine(a.out_val, a.out_grad, b->d_coef, b->offset, b->n_nets, n_sets, b->n_params, obj,
                       grad ? gobj : nullptr, st);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "combine launch");
    }
  }
  return TN_OK;
}

int batch_contract(tn_batch *b, const double *params, int n_sets, double *out, double *obj, void *stream) {
  return run_batch(b, false, params, n_sets, out, obj, nullptr, nullptr, (hipStream_t)stream);
}

int batch_grad(tn_batch *b, const double *params, int n_sets, double *out, double *obj, double *grad, double *gnet,
               void *stream) {
  return run_batch(b, true, params, n_sets, out, obj, grad, gnet, (hipStream_t)stream);
}

int batch_run_graph(tn_batch *b, int with_grad, const double *params, int n_sets, double *out, double *obj,
                    double *grad, double *grad_net, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!st) {
    set_error("tn_batch_run_graph: needs a non-default stream (graph capture)");
    return TN_EINVAL;
  }
  GraphCache &g = b->gc;
  bool hit = g.exec && g.with_grad == with_grad && g.n_sets == n_sets && g.params == params && g.out == out &&
             g.obj == obj && g.grad == grad && g.grad_net == grad_net && g.stream == st;
  if (!hit) {
    g.clear();
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    b->capturing = true;
    int rc = run_batch(b, with_grad != 0, params, n_sets, out, obj, grad, with_grad ? grad_net : nullptr, st);
    b->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != TN_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    g.graph = graph;
    HIPCHK(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    g.with_grad = with_grad;
    g.n_sets = n_sets;
    g.params = params;
    g.out = out;
    g.obj = obj;
    g.grad = grad;
    g.grad_net = grad_net;
    g.stream = st;
  }
  hipError_t e = hipGraphLaunch(g.exec, st);
  if (e != hipSuccess) {
    b->poisoned = true;
    return hip_fail(e, "hipGraphLaunch");
  }
  return TN_OK;
}

// Autotuner. (1) Fused executor: time the forward+adjoint pass with each
// workgroup size and keep the fastest. (2) Level executor: for every shape
// class of MFMA-eligible ops, time the matrix-core kernel against the thin
// kernel on scratch operands of that shape and keep the faster. Decisions
// live in the batch (and, with cache_path, in a text file of
// "key value" lines that later batches read first).
// Shortest of `reps` runs of fn (after one warm-up run), each between its
// own pair of events: robust to the occasional delayed launch.
static float time_ms(hipStream_t st, int reps, const std::function<int()> &fn, int &rc) {
  reps = std::max(1, reps);
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  rc = TN_OK;
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = TN_EDEVICE;
  float best = 0.f;
  if (rc == TN_OK && (rc = fn()) == TN_OK) {  // warm-up
    for (int i = 0; i < reps && rc == TN_OK; ++i) {
      (void)hipEventRecord(ev[2 * i], st);
      rc = fn();
      (void)hipEventRecord(ev[2 * i + 1], st);
    }
    if (rc == TN_OK && hipEventSynchronize(ev[2 * reps - 1]) == hipSuccess) {
      for (int i = 0; i < reps; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess && (i == 0 || ms < best)) best = ms;
      }
    }
  }
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  return best;
}

static std::map<std::string, int> read_cache(const char *path) {
  std::map<std::string, int> m;
  if (!path) return m;
  FILE *f = std::fopen(path, "r");
  if (!f) return m;
  char key[256];
  int v;
  while (std::fscanf(f, "%255s %d", key, &v) == 2) m[key] = v;
  std::fclose(f);
  return m;
}

static void write_cache(const char *path, const std::map<std::string, int> &add) {
  if (!path) return;
  auto m = read_cache(path);
  for (auto &kv : add) m[kv.first] = kv.second;
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  for (auto &kv : m) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
  std::fclose(f);
}

static std::string fused_key(const tn_batch *b) {
  return "fused_block:" + std::to_string(b->dtype) + ":" + std::to_string(b->hp.n_programs) + ":" +
         std::to_string(b->hp.ops.size()) + ":" + std::to_string(b->task_net.size());
}

int batch_autotune(tn_batch *b, const double *params, int n_sets, int reps, const char *cache_path, void *stream) {
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  if ((!params && b->n_params > 0) || n_sets < 1 || n_sets > b->max_sets) {
    set_error("tn_batch_autotune: n_sets out of range or params NULL");
    return TN_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  reps = std::max(1, reps);
  std::map<std::string, int> found;
  int rc = TN_OK;
  b->gc.clear();
  // (1) fused executor: adjoint programs by workgroup size or sets per wave,
  // then forward programs by sets per wave
  if (!b->task_net.empty()) {
    auto relayout = [&] { return (rc = layout_lds(b, 0)) == TN_OK && (rc = layout_lds(b, 1)) == TN_OK; };
    float best = 0.f, best_single = 0.f;
    int best_spw = b->spw[1], best_block = b->block, single_block = b->block;
    for (int cand : {64, 128, 256, -2, -4}) {
      if (cand < 0 && (b->max_sets == 1 || !sets_fit(b, -cand, b->fused_budget, 1))) continue;
      b->spw[1] = cand < 0 ? -cand : 1;
      if (cand > 0) b->block = cand;
      if (!relayout()) return rc;
      float ms = time_ms(st, reps, [&] { return run_batch(b, true, params, n_sets, nullptr, nullptr, nullptr, nullptr, st); },
                         rc);
      if (rc != TN_OK) return rc;
      if (best == 0.f || ms < best) {
        best = ms;
        best_spw = b->spw[1];
        best_block = b->block;
      }
      if (cand > 0 && (best_single == 0.f || ms < best_single)) {
        best_single = ms;
        single_block = cand;
      }
    }
    b->spw[1] = best_spw;
    b->block = best_spw > 1 ? single_block : best_block;
    best = 0.f;
    int best_fwd = b->spw[0];
    for (int S : {1, 2, 4}) {
      if (S > 1 && (b->max_sets == 1 || !sets_fit(b, S, b->fused_budget, 0))) continue;
      b->spw[0] = S;
      if (!relayout()) return rc;
      float ms = time_ms(st, reps, [&] { return run_batch(b, false, params, n_sets, nullptr, nullptr, nullptr, nullptr, st); },
                         rc);
      if (rc != TN_OK) return rc;
      if (best == 0.f || ms < best) {
        best = ms;
        best_fwd = S;
      }
    }
    b->spw[0] = best_fwd;
    if (!relayout()) return rc;
    const std::string suffix = fused_key(b).substr(12);
    found[fused_key(b)] = b->block;
    found["sets_per_wave:" + suffix] = b->spw[1];
    found["sets_per_wave_fwd:" + suffix] = b->spw[0];
  }
  // (2) large level ops: MFMA vs thin per shape class
  std::map<std::string, const DOp *> classes;
  for (const LevelNet &ln : b->level)
    for (int v = 0; v < 2; ++v)
      for (int o = 0; o < ln.n_ops[v]; ++o) {
        const DOp &op = b->hp.ops[ln.op_begin[v] + o];
        if (mfma_eligible(b->dtype, op)) classes.emplace(shape_class(b->dtype, op, b->mfma_prec), &op);
      }
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  for (auto &kv : classes) {
    DOp op = *kv.second;
    const int64_t nx = (int64_t)1 << (op.nFX + op.nS), ny = (int64_t)1 << (op.nS + op.nFY);
    const int64_t nz = (int64_t)1 << (op.nFX + op.nFY);
    // as many parameter vectors as the pass has (the launch shapes of the
    // real run), within 2^28 elements of scratch
    const int sets_t = (int)std::max<int64_t>(1, std::min<int64_t>(n_sets, ((int64_t)1 << 28) / (nx + ny + nz)));
    void *buf = nullptr;
    if (hipMalloc(&buf, (size_t)(nx + ny + nz) * sets_t * eb) != hipSuccess) {
      (void)hipGetLastError();
      continue;  // no room to tune this class: keep the default
    }
    HIPCHK(hipMemset(buf, 0, (size_t)(nx + ny + nz) * sets_t * eb));
    op.x = 0;
    op.y = (int32_t)nx;
    op.z = (int32_t)(nx + ny);
    LevelArgs la{};
    la.arena = buf;
    la.stride = nx + ny + nz;
    la.n_sets = sets_t;
    int rc1 = TN_OK, rc2 = TN_OK;
    float t_mfma = time_ms(st, reps, [&] { return mfma_contract(la, op, b->d_tabs + op.tab, b->mfma_prec, st) == hipSuccess ? TN_OK : TN_EDEVICE; }, rc1);
    // the thin kernel is not a candidate for large products (2^24 and more
    // complex multiply-adds per parameter vector): the matrix cores win there
    float t_thin = 1e30f;
    if (op.nFX + op.nS + op.nFY < 24)
      t_thin = time_ms(st, reps, [&] { return level_op(b->dtype, la, op, b->d_tabs, 0, st) == hipSuccess ? TN_OK : TN_EDEVICE; }, rc2);
    (void)hipFree(buf);
    if (rc1 != TN_OK || rc2 != TN_OK) {
      b->poisoned = true;
      set_error("tn_batch_autotune: launch failed");
      return TN_EDEVICE;
    }
    b->use_mfma[kv.first] = t_mfma <= t_thin ? 1 : 0;
    found["mfma:" + kv.first] = b->use_mfma[kv.first];
    // measured times (ns, at sets_t angle sets), recorded for inspection only
    found["time_ns_mfma:" + kv.first + ":sets" + std::to_string(sets_t)] = (int)std::min(2e9f, t_mfma * 1e6f);
    if (t_thin < 1e29f)
      found["time_ns_thin:" + kv.first + ":sets" + std::to_string(sets_t)] = (int)std::min(2e9f, t_thin * 1e6f);
  }
  write_cache(cache_path, found);
  return build_level_items(b);
}

int batch_kernel_timing(tn_batch *b, int enable) {
  b->timing = enable != 0;
  if (!b->timing) drop_timing_events(b);
  return TN_OK;
}

int batch_kernel_time(tn_batch *b, int *n, double *total_ms) {
  double sum = 0.0;
  int cnt = 0;
  hipError_t e = hipSuccess;
  for (auto &pr : b->tev) {
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e == hipSuccess) {
      sum += ms;
      ++cnt;
    }
  }
  drop_timing_events(b);
  if (e != hipSuccess) return hip_fail(e, "tn_batch_kernel_time");
  *n = cnt;
  *total_ms = sum;
  return TN_OK;
}

int batch_set_precision(tn_batch *b, int prec) {
  const bool ok = b->dtype == TN_C128 ? prec == TN_MFMA_FP64 : (prec == TN_MFMA_FP32 || prec == TN_MFMA_BF16X3);
  if (!ok) {
    set_error("tn_batch_set_precision: precision not available for this batch's dtype");
    return TN_EINVAL;
  }
  b->mfma_prec = prec;
  return build_level_items(b);
}

// Apply cached autotuner decisions (no timing).
int batch_apply_cache(tn_batch *b, const char *cache_path) {
  auto m = read_cache(cache_path);
  auto it = m.find(fused_key(b));
  if (it != m.end() && (it->second == 64 || it->second == 128 || it->second == 256) && !b->task_net.empty()) {
    b->block = it->second;
    const std::string suffix = fused_key(b).substr(12);
    for (int v = 0; v < 2; ++v) {
      auto is = m.find((v == 0 ? "sets_per_wave_fwd:" : "sets_per_wave:") + suffix);
      if (is != m.end() &&
          (is->second == 1 || ((is->second == 2 || is->second == 4) && sets_fit(b, is->second, b->fused_budget, v))))
        b->spw[v] = is->second;
    }
    int rc;
    if ((rc = layout_lds(b, 0)) != TN_OK || (rc = layout_lds(b, 1)) != TN_OK) return rc;
  }
  for (auto &kv : m)
    if (kv.first.rfind("mfma:", 0) == 0) b->use_mfma[kv.first.substr(5)] = kv.second;
  return build_level_items(b);
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
  s->n_level_bins = (int32_t)b->lbins.size();
  s->n_level_chunked = (int32_t)b->lsolo.size();
  for (int v = 0; v < 2; ++v) {
    int64_t n = 0;
    for (const LevelBin &bn : b->lbins) {
      n += 2 * (int64_t)bn.lv.size();  // set-up and outputs
      for (const LevelBin::Step &stp : bn.steps[v]) {
        n += (stp.nt > 0) + stp.ng + (stp.nr > 0);
        for (int q = stp.o0; q < stp.o0 + stp.no; ++q) {
          const LevelNet &ln = b->level[bn.lv[bn.other[v][q]]];
          n += b->hp.ops[ln.op_begin[v] + (int)(&stp - bn.steps[v].data())].type == OP_SCALAR ? 2 : 1;
        }
      }
    }
    for (int l : b->lsolo) {
      const LevelNet &ln = b->level[l];
      int64_t per = 2;
      for (int o = 0; o < ln.n_ops[v]; ++o) per += b->hp.ops[ln.op_begin[v] + o].type == OP_SCALAR ? 2 : 1;
      n += per * ((b->max_sets + ln.chunk - 1) / ln.chunk);
    }
    (v == 0 ? s->level_launches_fwd : s->level_launches_grad) = (int32_t)std::min<int64_t>(n, INT32_MAX);
    int32_t ns = 0;
    for (const LevelBin &bn : b->lbins)
      for (const LevelBin::Step &stp : bn.steps[v]) ns += stp.nr;
    (v == 0 ? s->level_split_fwd : s->level_split_grad) = ns;
  }
  s->n_programs = b->hp.n_programs;
  s->fused_block = b->block;
  s->sets_per_wave_fwd = b->spw[0];
  s->sets_per_wave_grad = b->spw[1];
  s->rec_only = (rec_only(b, 0) ? 1 : 0) | (rec_only(b, 1) ? 2 : 0);
  s->lds_bytes_fwd = b->lds_fwd;
  s->lds_bytes_grad = b->lds_grad;
  s->flops_fwd = b->flops_fwd;
  s->bytes_fwd = b->bytes_fwd;
  s->flops_grad = b->flops_grad;
  s->bytes_grad = b->bytes_grad;
  return TN_OK;
}

int stream_sync(void *stream) {
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return TN_OK;
}

void batch_free(tn_batch *b) {
  if (!b) return;
  free_batch_dev(b);
  delete b;
}

// Single-network plain path: a cached one-network batch; host parameters in,
// host scalar out; synchronises the stream.
// Device state of the one-network path: a one-network batch and a pinned,
// device-mapped host block [params | value (2) | gradient] that the binding
// kernel reads and the fused kernel writes directly (no copies per call).
struct NetDev {
  tn_batch *b = nullptr;
  double *h_io = nullptr;                          // host view
  double *d_params = nullptr, *d_out = nullptr, *d_grad = nullptr;  // device views of h_io
};

static int net_dev(Net &net, NetDev *&nd) {
  nd = reinterpret_cast<NetDev *>(net.dev);
  if (nd) return TN_OK;
  std::unique_ptr<NetDev> n(new NetDev());
  tn_net *self = reinterpret_cast<tn_net *>(&net);
  int rc = batch_create(&self, 1, nullptr, 0.0, 1, &n->b);
  if (rc != TN_OK) return rc;
  hipError_t e;
  const size_t np = (size_t)std::max(1, net.n_params);
  double *dv = nullptr;
  if ((e = hipHostMalloc((void **)&n->h_io, (2 * np + 2) * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent)) !=
          hipSuccess ||
      (e = hipHostGetDevicePointer((void **)&dv, n->h_io, 0)) != hipSuccess) {
    if (n->h_io) (void)hipHostFree(n->h_io);
    batch_free(n->b);
    return hip_fail(e, "hipHostMalloc");
  }
  n->d_params = dv;
  n->d_out = dv + np;
  n->d_grad = dv + np + 2;
  nd = n.release();
  net.dev = nd;
  return TN_OK;
}

void net_dev_free(Net &net) {
  NetDev *nd = reinterpret_cast<NetDev *>(net.dev);
  if (!nd) return;
  batch_free(nd->b);
  if (nd->h_io) (void)hipHostFree(nd->h_io);
  delete nd;
  net.dev = nullptr;
}

int net_contract(Net &net, const double *params, double *out, double *value, double *grad, void *stream) {
  if (net.poisoned) {
    set_error("network poisoned by an earlier device error");
    return TN_ESTATE;
  }
  if (!net.has_order) {
    set_error("no contraction order set");
    return TN_EORDER;
  }
  if (net.n_params > 0 && !params) {
    set_error("params is NULL");
    return TN_EINVAL;
  }
  NetDev *nd;
  int rc = net_dev(net, nd);
  if (rc != TN_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  auto bad = [&](hipError_t e, const char *w) {
    net.poisoned = true;
    return hip_fail(e, w);
  };
  hipError_t e;
  // the previous call on this network has finished (it synchronised), so
  // the mapped block is free to rewrite
  const size_t np = (size_t)std::max(1, net.n_params);
  if (net.n_params > 0) std::memcpy(nd->h_io, params, net.n_params * sizeof(double));
  const bool g = grad != nullptr;
  rc = g ? batch_grad(nd->b, nd->d_params, 1, nd->d_out, nullptr, nullptr, nd->d_grad, st)
         : batch_contract(nd->b, nd->d_params, 1, nd->d_out, nullptr, st);
  if (rc != TN_OK) {
    net.poisoned = rc == TN_EDEVICE;
    return rc;
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return bad(e, "hipStreamSynchronize");
  const double *h = nd->h_io + np;
  if (g && net.n_params > 0) std::memcpy(grad, h + 2, net.n_params * sizeof(double));
  if (out) {
    out[0] = h[0];
    out[1] = h[1];
  }
  if (value) *value = h[0];
  return TN_OK;
}

int net_bind(Net &net, const double *params, int n_sets, void *dst, int64_t *per_set, void *stream) {
  int64_t total = 0;
  std::vector<DParam> dp;
  for (auto &pt : net.ptensors) {
    DParam d{};
    d.kind = pt.kind;
    d.param = pt.param;
    d.folded = pt.folded;
    d.diag = pt.diag;
    d.bits = pt.bits;
    d.off = (int32_t)total;
    d.coeff = pt.coeff;
    dp.push_back(d);
    total += (int64_t)1 << pt.bits;
  }
  if (per_set) *per_set = total;
  if (!dst) return TN_OK;
  if (!params || n_sets < 1) {
    set_error("tn_bind_params: bad arguments");
    return TN_EINVAL;
  }
  if (dp.empty()) return TN_OK;
  DParam *d_dp = nullptr;
  HIPCHK(dalloc(&d_dp, dp.size()));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d_dp, dp.data(), dp.size() * sizeof(DParam), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_bind(net.dtype, d_dp, (int)dp.size(), params, net.n_params, n_sets, (int)total, dst, nullptr, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_dp);
  if (e != hipSuccess) return hip_fail(e, "tn_bind_params");
  return TN_OK;
}

}  // namespace qtn
