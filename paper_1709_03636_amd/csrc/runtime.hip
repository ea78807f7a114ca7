// Batch runtime: turns compiled network programs into device arrays, lays
// out executor memory, launches the kernels and captures HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <numeric>

#include "device.hpp"
#include "internal.hpp"

namespace qtn {

hipError_t launch_fused(int dtype, int block, const FusedArgs &a, int grid, int lds_bytes, hipStream_t st);
const void *fused_kernel_ptr(int dtype, int block);
hipError_t launch_combine(const double *val, const double *gnet, const double *coef, double offset, int n_nets,
                          int n_sets, int n_params, double *obj, double *grad, hipStream_t st);
hipError_t launch_bind(int dtype, const DParam *ptens, int n_ptens, const double *params, int n_params, int n_sets,
                       int per_set, void *dst, hipStream_t st);


static constexpr int kLdsCap = 160 * 1024;

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

struct HostProgram {
  std::vector<DNet> nets_fwd, nets_grad;
  std::vector<DOp> ops;
  std::vector<int32_t> tabs;
  std::vector<double> consts;  // interleaved, converted to the dtype at upload
  std::vector<DParam> ptens;
  int max_mem_fwd = 0, max_mem_grad = 0, max_comp = 0;
};

// Append the fused programs (forward and forward+adjoint) of one network.
static int append_fused(const Net &net, HostProgram &hp, std::string &why) {
  const Plan &p = net.gplan;
  const int L = p.n_leaves;
  // leaf region: constants then parametric tensors
  std::vector<int64_t> coff(net.consts.size()), poff(net.ptensors.size());
  int64_t pos = 0;
  const int const_begin = (int)(hp.consts.size() / 2);
  for (size_t c = 0; c < net.consts.size(); ++c) {
    coff[c] = pos;
    for (auto &z : net.consts[c]) {
      hp.consts.push_back(z.real());
      hp.consts.push_back(z.imag());
    }
    pos += (int64_t)net.consts[c].size();
  }
  const int n_const = (int)pos;
  const int ptens_begin = (int)hp.ptens.size();
  for (size_t t = 0; t < net.ptensors.size(); ++t) {
    const ParamTensor &pt = net.ptensors[t];
    poff[t] = pos;
    DParam d{};
    d.kind = pt.kind;
    d.param = pt.param;
    d.folded = pt.folded;
    d.bits = pt.bits;
    d.off = (int32_t)pos;
    d.coeff = pt.coeff;
    hp.ptens.push_back(d);
    pos += (int64_t)1 << pt.bits;
  }
  const int64_t leaf_region = pos;
  auto leaf_off = [&](int v) -> int64_t {
    int src = net.leaves[v].src;
    return src >= 0 ? coff[src] : poff[-src - 1];
  };
  for (int variant = 0; variant < 2; ++variant) {
    const int n_ops = variant == 0 ? p.n_fwd_ops : (int)p.ops.size();
    std::vector<int64_t> off;
    int64_t arena = layout_buffers(p, n_ops, off);
    int64_t mem = leaf_region + arena;
    if (mem * net.elem_bytes() > kLdsCap) {
      why = "needs " + std::to_string(mem * net.elem_bytes()) + " bytes of LDS";
      return TN_ENOMEM;
    }
    auto boff = [&](int v) -> int32_t { return (int32_t)(v < L ? leaf_off(v) : leaf_region + off[v]); };
    DNet dn{};
    dn.op_begin = (int32_t)hp.ops.size();
    dn.n_ops = n_ops;
    dn.n_comp = p.n_components;
    dn.mem_elems = (int32_t)mem;
    dn.const_begin = const_begin;
    dn.n_const = n_const;
    dn.ptens_begin = ptens_begin;
    dn.n_ptens = (int32_t)net.ptensors.size();
    for (int i = 0; i < n_ops; ++i) {
      const Op &op = p.ops[i];
      DOp d{};
      d.type = op.type;
      d.nFX = op.nFX;
      d.nS = op.nS;
      d.nFY = op.nFY;
      d.maskX = op.maskX_F;
      d.maskY = op.maskY_F;
      d.tab = (int32_t)hp.tabs.size();
      hp.tabs.insert(hp.tabs.end(), op.tab.begin(), op.tab.end());
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
        d.aux0 = ptens_begin + op.aux0;
        d.aux1 = op.aux1;
      }
      hp.ops.push_back(d);
    }
    (variant == 0 ? hp.nets_fwd : hp.nets_grad).push_back(dn);
    int &mx = variant == 0 ? hp.max_mem_fwd : hp.max_mem_grad;
    mx = std::max(mx, (int)mem);
  }
  hp.max_comp = std::max(hp.max_comp, p.n_components);
  return TN_OK;
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
  const void *params = nullptr, *out = nullptr, *obj = nullptr, *grad = nullptr;
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
  double offset = 0;
  std::vector<double> coef;
  qtn::HostProgram hp;
  std::vector<int32_t> task_net;
  // device
  qtn::DNet *d_nets_fwd = nullptr, *d_nets_grad = nullptr;
  qtn::DOp *d_ops = nullptr;
  int32_t *d_tabs = nullptr, *d_task_net = nullptr;
  void *d_consts = nullptr;
  qtn::DParam *d_ptens = nullptr;
  int *d_counter = nullptr;
  double *d_val = nullptr, *d_gnet = nullptr, *d_coef = nullptr;
  int lds_fwd = 0, lds_grad = 0, grid_fwd = 0, grid_grad = 0;
  int scratch_off[2], scal_off[2], gacc_off[2], red_off[2];
  double flops_fwd = 0, bytes_fwd = 0, flops_grad = 0, bytes_grad = 0;
  bool poisoned = false;
  qtn::GraphCache gc;
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

static void free_batch_dev(tn_batch *b) {
  b->gc.clear();
  void *ptrs[] = {b->d_nets_fwd, b->d_nets_grad, b->d_ops, b->d_tabs, b->d_task_net, b->d_consts,
                  b->d_ptens, b->d_counter, b->d_val, b->d_gnet, b->d_coef};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
}

static int layout_lds(tn_batch *b, int variant) {
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const int mem = variant == 0 ? b->hp.max_mem_fwd : b->hp.max_mem_grad;
  auto al = [](int x) { return (x + 15) & ~15; };
  int o = al(mem * eb);
  b->scratch_off[variant] = o;
  o = al(o + b->block * eb);
  b->scal_off[variant] = o;
  o = al(o + std::max(1, b->hp.max_comp) * 16);
  b->gacc_off[variant] = o;
  o = al(o + std::max(1, b->n_params) * 8);
  b->red_off[variant] = o;
  o = al(o + 16 * 8);
  if (o > kLdsCap) {
    set_error("fused executor: LDS layout of " + std::to_string(o) + " bytes exceeds 160 KiB");
    return TN_ENOMEM;
  }
  (variant == 0 ? b->lds_fwd : b->lds_grad) = o;
  int per_cu = 0;
  const void *k = fused_kernel_ptr(b->dtype, b->block);
  if (o > 64 * 1024) HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, o));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, b->block, o));
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int grid = std::max(1, per_cu) * std::max(1, cus);
  (variant == 0 ? b->grid_fwd : b->grid_grad) = grid;
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
  b->n_nets = n_nets;
  b->n_params = n0->n_params;
  b->max_sets = max_sets;
  b->offset = offset;
  b->coef.assign(n_nets, 0.0);
  if (coef) std::copy(coef, coef + n_nets, b->coef.begin());
  std::vector<double> cost(n_nets);
  for (int i = 0; i < n_nets; ++i) {
    const Net *n = reinterpret_cast<const Net *>(nets[i]);
    std::string why;
    int rc = append_fused(*n, b->hp, why);
    if (rc != TN_OK) {
      set_error("tn_batch_create: network " + std::to_string(i) + " does not fit the fused executor (" + why + ")");
      return rc;
    }
    cost[i] = n->gplan.flops + n->gplan.flops_grad + 1e3 * n->gplan.ops.size();
    b->flops_fwd += n->gplan.flops;
    b->bytes_fwd += n->gplan.bytes;
    b->flops_grad += n->gplan.flops_grad;
    b->bytes_grad += n->gplan.bytes_grad;
  }
  // expensive networks first (longest-processing-time order for the work queue)
  b->task_net.resize(n_nets);
  std::iota(b->task_net.begin(), b->task_net.end(), 0);
  std::stable_sort(b->task_net.begin(), b->task_net.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  // block size: enough threads for the typical op, few idle lanes
  int maxbits = 0;
  for (int i = 0; i < n_nets; ++i) maxbits = std::max(maxbits, reinterpret_cast<const Net *>(nets[i])->gplan.peak_bits);
  b->block = maxbits <= 6 ? 64 : (maxbits <= 9 ? 128 : 256);
  int rc;
  if ((rc = layout_lds(b.get(), 0)) != TN_OK) return rc;
  if ((rc = layout_lds(b.get(), 1)) != TN_OK) return rc;

  tn_batch *B = b.get();
  auto fail = [&](hipError_t e, const char *w) {
    free_batch_dev(B);
    return hip_fail(e, w);
  };
  hipError_t e;
  const HostProgram &hp = b->hp;
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  if ((e = dalloc(&b->d_nets_fwd, hp.nets_fwd.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_nets_grad, hp.nets_grad.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_ops, hp.ops.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_tabs, hp.tabs.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_task_net, b->task_net.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc((char **)&b->d_consts, hp.consts.size() / 2 * eb)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_ptens, hp.ptens.size())) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_counter, 2)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMemset(b->d_counter, 0, 2 * sizeof(int))) != hipSuccess) return fail(e, "hipMemset");
  if ((e = dalloc(&b->d_val, (size_t)n_nets * max_sets * 2)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_gnet, (size_t)n_nets * max_sets * std::max(1, b->n_params))) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = dalloc(&b->d_coef, (size_t)n_nets)) != hipSuccess) return fail(e, "hipMalloc");
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
      {b->d_task_net, b->task_net.data(), b->task_net.size() * sizeof(int32_t)},
      {b->d_consts, csrc, hp.consts.size() / 2 * eb},
      {b->d_ptens, hp.ptens.data(), hp.ptens.size() * sizeof(DParam)},
      {b->d_coef, b->coef.data(), b->coef.size() * sizeof(double)},
  };
  for (auto &u : ups)
    if (u.n && (e = hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "hipMemcpy");
  *out = b.release();
  return TN_OK;
}

static int run_batch(tn_batch *b, bool grad, const double *params, int n_sets, double *out, double *obj, double *gobj,
                     double *gnet_out, hipStream_t st) {
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  if (!params || n_sets < 1 || n_sets > b->max_sets) {
    set_error("batch run: n_sets out of range or params NULL");
    return TN_EINVAL;
  }
  const int v = grad ? 1 : 0;
  FusedArgs a{};
  a.nets = grad ? b->d_nets_grad : b->d_nets_fwd;
  a.ops = b->d_ops;
  a.tabs = b->d_tabs;
  a.consts = b->d_consts;
  a.ptens = b->d_ptens;
  a.params = params;
  a.task_net = b->d_task_net;
  a.counter = b->d_counter;
  // network-major output; the internal buffer is used when the caller's
  // layout would not match or no pointer is given
  a.out_val = out ? out : b->d_val;
  a.out_grad = gnet_out ? gnet_out : b->d_gnet;
  a.n_params = b->n_params;
  a.n_sets = n_sets;
  a.n_tasks = b->n_nets * n_sets;
  a.scratch_off = b->scratch_off[v];
  a.scal_off = b->scal_off[v];
  a.gacc_off = b->gacc_off[v];
  a.red_off = b->red_off[v];
  a.with_grad = grad ? 1 : 0;
  const int grid = std::min(grad ? b->grid_grad : b->grid_fwd, a.n_tasks);
  hipError_t e = launch_fused(b->dtype, b->block, a, grid, grad ? b->lds_grad : b->lds_fwd, st);
  if (e != hipSuccess) {
    b->poisoned = true;
    return hip_fail(e, "fused executor launch");
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
                    double *grad, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!st) {
    set_error("tn_batch_run_graph: needs a non-default stream (graph capture)");
    return TN_EINVAL;
  }
  GraphCache &g = b->gc;
  bool hit = g.exec && g.with_grad == with_grad && g.n_sets == n_sets && g.params == params && g.out == out &&
             g.obj == obj && g.grad == grad && g.stream == st;
  if (!hit) {
    g.clear();
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = run_batch(b, with_grad != 0, params, n_sets, out, obj, grad, nullptr, st);
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
    g.stream = st;
  }
  hipError_t e = hipGraphLaunch(g.exec, st);
  if (e != hipSuccess) {
    b->poisoned = true;
    return hip_fail(e, "hipGraphLaunch");
  }
  return TN_OK;
}

int batch_info(const tn_batch *b, tn_batch_stats *s) {
  std::memset(s, 0, sizeof(*s));
  s->n_nets = b->n_nets;
  s->n_fused = b->n_nets;
  s->n_level = 0;
  s->n_levels = 0;
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
struct NetDev {
  tn_batch *b = nullptr;
  double *d_params = nullptr, *d_out = nullptr, *d_grad = nullptr;
};

static int net_dev(Net &net, NetDev *&nd) {
  nd = reinterpret_cast<NetDev *>(net.dev);
  if (nd) return TN_OK;
  std::unique_ptr<NetDev> n(new NetDev());
  tn_net *self = reinterpret_cast<tn_net *>(&net);
  int rc = batch_create(&self, 1, nullptr, 0.0, 1, &n->b);
  if (rc != TN_OK) return rc;
  hipError_t e;
  if ((e = dalloc(&n->d_params, std::max(1, net.n_params))) != hipSuccess ||
      (e = dalloc(&n->d_out, 2)) != hipSuccess || (e = dalloc(&n->d_grad, std::max(1, net.n_params))) != hipSuccess) {
    batch_free(n->b);
    return hip_fail(e, "hipMalloc");
  }
  nd = n.release();
  net.dev = nd;
  return TN_OK;
}

void net_dev_free(Net &net) {
  NetDev *nd = reinterpret_cast<NetDev *>(net.dev);
  if (!nd) return;
  batch_free(nd->b);
  for (void *p : {(void *)nd->d_params, (void *)nd->d_out, (void *)nd->d_grad})
    if (p) (void)hipFree(p);
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
  if (net.n_params > 0 &&
      (e = hipMemcpyAsync(nd->d_params, params, net.n_params * sizeof(double), hipMemcpyHostToDevice, st)) != hipSuccess)
    return bad(e, "hipMemcpyAsync");
  const bool g = grad != nullptr;
  rc = g ? batch_grad(nd->b, nd->d_params, 1, nd->d_out, nullptr, nullptr, nd->d_grad, st)
         : batch_contract(nd->b, nd->d_params, 1, nd->d_out, nullptr, st);
  if (rc != TN_OK) {
    net.poisoned = rc == TN_EDEVICE;
    return rc;
  }
  double h[2];
  if ((e = hipMemcpyAsync(h, nd->d_out, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) return bad(e, "hipMemcpyAsync");
  if (g && net.n_params > 0 &&
      (e = hipMemcpyAsync(grad, nd->d_grad, net.n_params * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return bad(e, "hipMemcpyAsync");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return bad(e, "hipStreamSynchronize");
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
  if (e == hipSuccess) e = launch_bind(net.dtype, d_dp, (int)dp.size(), params, net.n_params, n_sets, (int)total, dst, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_dp);
  if (e != hipSuccess) return hip_fail(e, "tn_bind_params");
  return TN_OK;
}

}  // namespace qtn
