// Batch runtime: binds a batch's device workspace, uploads the planned
// arrays, launches the executors (angle binding, fused executor in LDS or on
// global-arena slots, the level executor's task executor or item launches,
// the combine)
// and captures HIP graphs. Planning lives in bplan.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>

#include "batch.hpp"
#include "device.hpp"
#include "internal.hpp"
#include "kargs.hpp"

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
hipError_t item_launch(int prec, const PItem &it, const LvlArgs &a, hipStream_t st);
hipError_t task_reset(const LvlArgs &a, hipStream_t st);
hipError_t task_run(int prec, const LvlArgs &a, int grid, hipStream_t st);
const void *task_kernel_ptr(int prec);

// --- device memory: the caller's allocator, or hipMalloc ----------------------------------------

static std::mutex g_alloc_mu;
static tn_alloc_fn g_alloc = nullptr;
static tn_free_fn g_free = nullptr;
static void *g_alloc_ctx = nullptr;

int set_allocator(tn_alloc_fn alloc, tn_free_fn release, void *ctx) {
  if ((alloc == nullptr) != (release == nullptr)) {
    set_error("tn_set_allocator: give both functions or neither");
    return TN_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = release;
  g_alloc_ctx = ctx;
  return TN_OK;
}

// Device memory of `bytes` bytes (at least 1) from the registered allocator
// or hipMalloc; nullptr on failure (message set).
void *dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 1;
  tn_alloc_fn fa;
  void *ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    fa = g_alloc;
    ctx = g_alloc_ctx;
  }
  void *p = nullptr;
  if (fa) {
    p = fa((uint64_t)bytes, ctx);
    if (!p) set_error("device allocator returned NULL for " + std::to_string(bytes) + " bytes");
    return p;
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return nullptr;
  }
  return p;
}

void dev_free(void *p) {
  if (!p) return;
  tn_free_fn ff;
  void *ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    ff = g_free;
    ctx = g_alloc_ctx;
  }
  if (ff) ff(p, ctx);
  else (void)hipFree(p);
}

static int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return TN_EDEVICE;
}

#define HIPCHK(call)                                    \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hip_fail(_e, #call);   \
  } while (0)

static inline hipStream_t hs(void *p) { return (hipStream_t)p; }
static inline hipEvent_t he(void *p) { return (hipEvent_t)p; }

template <typename T>
static T *ws_ptr(const tn_batch *b, int k) {
  return reinterpret_cast<T *>(b->d_ws + b->ws.off[k]);
}

// Array k of a workspace at ws (the bound one, or the static scratch).
template <typename T>
static T *wsp(char *ws, const tn_batch *b, int k) {
  return reinterpret_cast<T *>(ws + b->ws.off[k]);
}

static void drop_timing_events(tn_batch *b) {
  for (auto &v : b->tev) {
    for (auto &pr : v) {
      (void)hipEventDestroy(he(pr.first));
      (void)hipEventDestroy(he(pr.second));
    }
    v.clear();
  }
}

// Kernel timing: an event pair around one executor's launch on its stream
// (eager runs in the bound workspace only; at most 4096 pending pairs each).
struct TimedLaunch {
  hipEvent_t t0 = nullptr, t1 = nullptr;
};

static TimedLaunch timing_begin(tn_batch *b, int kind, bool own_ws, hipStream_t s) {
  TimedLaunch t;
  if (!b->timing || b->capturing || own_ws || b->tev[kind].size() >= 4096) return t;
  if (hipEventCreate(&t.t0) != hipSuccess) return TimedLaunch{};
  if (hipEventCreate(&t.t1) != hipSuccess || hipEventRecord(t.t0, s) != hipSuccess) {
    (void)hipEventDestroy(t.t0);
    if (t.t1) (void)hipEventDestroy(t.t1);
    return TimedLaunch{};
  }
  return t;
}

static void timing_end(tn_batch *b, int kind, hipStream_t s, hipError_t launched, TimedLaunch &t) {
  if (!t.t0) return;
  if (launched == hipSuccess && hipEventRecord(t.t1, s) == hipSuccess) {
    b->tev[kind].emplace_back(t.t0, t.t1);
  } else {
    (void)hipEventDestroy(t.t0);
    (void)hipEventDestroy(t.t1);
  }
  t = TimedLaunch{};
}

static void graph_clear(tn_batch *b) {
  if (b->gc.exec) (void)hipGraphExecDestroy((hipGraphExec_t)b->gc.exec);
  if (b->gc.graph) (void)hipGraphDestroy((hipGraph_t)b->gc.graph);
  b->gc.exec = b->gc.graph = nullptr;
}

static void free_device(tn_batch *b) {
  if (b->d_ws) (void)hipDeviceSynchronize();  // no kernel may still use the workspace
  graph_clear(b);
  drop_timing_events(b);
  if (b->ev_fork) (void)hipEventDestroy(he(b->ev_fork));
  b->ev_fork = nullptr;
  for (int i = 0; i < 2; ++i) {
    if (b->ev_join[i]) (void)hipEventDestroy(he(b->ev_join[i]));
    if (b->side[i]) (void)hipStreamDestroy(hs(b->side[i]));
    b->ev_join[i] = nullptr;
    b->side[i] = nullptr;
  }
  if (b->ws_owned) dev_free(b->d_ws);
  b->d_ws = nullptr;
  b->ws_owned = false;
  b->uploaded = false;
}

// 64-lane workgroups whose programs have a lane record for every op run a
// kernel instance without the descriptor path (fewer registers live across
// the op loop).
static bool rec_only(const tn_batch *b, int variant) { return b->block == kRecLanes && !b->hp.generic[variant]; }

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
  }
  return TN_OK;
}


// Upload the task executor's items and networks (after planning or a change
// of matrix-core choices). Synchronous; never under capture.
static int upload_items(tn_batch *b) {
  HIPCHK(hipDeviceSynchronize());  // earlier launches may still read the old lists
  for (int v = 0; v < 2; ++v) {
    if ((int64_t)b->titems[v].size() > b->cap_titems[v]) {
      set_error("level plan larger than its workspace room");
      return TN_EINVAL;
    }
    if (!b->titems[v].empty())
      HIPCHK(hipMemcpy(ws_ptr<char>(b, v ? WsLayout::TITEMS1 : WsLayout::TITEMS0), b->titems[v].data(),
                       b->titems[v].size() * sizeof(PItem), hipMemcpyHostToDevice));
    if (!b->tnets[v].empty())
      HIPCHK(hipMemcpy(ws_ptr<char>(b, v ? WsLayout::TNETS1 : WsLayout::TNETS0), b->tnets[v].data(),
                       b->tnets[v].size() * sizeof(TNet), hipMemcpyHostToDevice));
  }
  if ((int64_t)b->trecs.size() > b->cap_trecs) {
    set_error("task-executor lane records larger than their workspace room");
    return TN_EINVAL;
  }
  if (!b->trecs.empty())
    HIPCHK(hipMemcpy(ws_ptr<char>(b, WsLayout::TRECS), b->trecs.data(), b->trecs.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
  b->items_dirty = false;
  graph_clear(b);
  return TN_OK;
}

// Workgroups of the task executor: as many as stay resident.
static int task_grid(tn_batch *b) {
  const int prec = b->dtype == TN_C128 ? TN_MFMA_FP64 : b->mfma_prec;
  if (b->task_grid > 0 && b->task_grid_prec == prec) return TN_OK;
  int dev = 0, cus = 0, per_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, task_kernel_ptr(prec), 256, 0));
  b->task_grid = std::max(1, per_cu) * std::max(1, cus);
  b->task_grid_prec = prec;
  return TN_OK;
}

static int upload_tables(tn_batch *b, char *ws, hipStream_t st, bool async, bool with_items);

// Bind the workspace: program arrays uploaded, launch shapes from the
// device's occupancy, side streams for the executors with work.
int batch_bind(tn_batch *b, void *ptr, int64_t bytes) {
  if (!ptr || bytes < b->ws.total) {
    set_error("tn_batch_set_workspace: needs " + std::to_string(b->ws.total) + " bytes of device memory");
    return TN_EINVAL;
  }
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  free_device(b);
  b->d_ws = static_cast<char *>(ptr);
  int rc = upload_tables(b, b->d_ws, nullptr, false, false);
  if (rc != TN_OK) return rc;
  // side streams only for the executors that have work (streams share the
  // few hardware queues: an idle stream could take a busy one's queue)
  const bool fused = !b->task_net.empty(), gmem = !b->gtask_net.empty(), lvl = !b->level.empty();
  if (fused + gmem + lvl >= 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->ev_fork = e;
    const bool need[2] = {gmem, lvl};
    for (int i = 0; i < 2; ++i) {
      if (!need[i]) continue;
      hipStream_t s;
      HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->side[i] = s;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->ev_join[i] = e;
    }
  }
  if ((rc = layout_lds(b, 0)) != TN_OK || (rc = layout_lds(b, 1)) != TN_OK || (rc = layout_gmem(b)) != TN_OK) return rc;
  b->uploaded = true;
  b->items_dirty = true;
  return upload_items(b);
}

// The program arrays into the workspace at ws (the task executor's lists
// only when with_items): synchronous copies, or, when async, copies ordered
// on st that read the batch's host arrays (which outlive the call).
static int upload_tables(tn_batch *b, char *ws, hipStream_t st, bool async, bool with_items) {
  const HostProgram &hp = b->hp;
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const void *csrc = b->dtype == TN_C64 ? (const void *)b->consts_f.data() : (const void *)hp.consts.data();
  struct Up { int k; const void *h; size_t n; } ups[] = {
      {WsLayout::NETS_FWD, hp.nets_fwd.data(), hp.nets_fwd.size() * sizeof(DNet)},
      {WsLayout::NETS_GRAD, hp.nets_grad.data(), hp.nets_grad.size() * sizeof(DNet)},
      {WsLayout::OPS, hp.ops.data(), hp.ops.size() * sizeof(DOp)},
      {WsLayout::TABS, hp.tabs.data(), hp.tabs.size() * sizeof(int32_t)},
      {WsLayout::RECS, hp.recs.data(), hp.recs.size() * sizeof(int32_t)},
      {WsLayout::SRECS0, hp.srecs[0].data(), hp.srecs[0].size() * sizeof(int32_t)},
      {WsLayout::SRECS1, hp.srecs[1].data(), hp.srecs[1].size() * sizeof(int32_t)},
      {WsLayout::TASK_NET, b->task_net.data(), b->task_net.size() * sizeof(int32_t)},
      {WsLayout::GTASK_NET, b->gtask_net.data(), b->gtask_net.size() * sizeof(int32_t)},
      {WsLayout::CONSTS, csrc, hp.consts.size() / 2 * eb},
      {WsLayout::PTENS, hp.ptens.data(), hp.ptens.size() * sizeof(DParam)},
      {WsLayout::SLOTS, hp.slots.data(), hp.slots.size() * sizeof(DParam)},
      {WsLayout::COEF, b->coef.data(), b->coef.size() * sizeof(double)},
      {WsLayout::TITEMS0, b->titems[0].data(), with_items ? b->titems[0].size() * sizeof(PItem) : 0},
      {WsLayout::TITEMS1, b->titems[1].data(), with_items ? b->titems[1].size() * sizeof(PItem) : 0},
      {WsLayout::TNETS0, b->tnets[0].data(), with_items ? b->tnets[0].size() * sizeof(TNet) : 0},
      {WsLayout::TNETS1, b->tnets[1].data(), with_items ? b->tnets[1].size() * sizeof(TNet) : 0},
      {WsLayout::TRECS, b->trecs.data(), with_items ? b->trecs.size() * sizeof(int32_t) : 0},
  };
  for (auto &u : ups) {
    if (!u.n) continue;
    if ((int64_t)u.n > b->ws.size[u.k]) {
      set_error("batch program larger than its workspace room");
      return TN_EINVAL;
    }
    if (async)
      HIPCHK(hipMemcpyAsync(wsp<char>(ws, b, u.k), u.h, u.n, hipMemcpyHostToDevice, st));
    else
      HIPCHK(hipMemcpy(wsp<char>(ws, b, u.k), u.h, u.n, hipMemcpyHostToDevice));
  }
  return TN_OK;
}

// A batch run without a bound workspace gets one from the allocator.
static int ensure_bound(tn_batch *b) {
  if (b->d_ws) return b->items_dirty ? upload_items(b) : TN_OK;
  void *p = dev_alloc((size_t)b->ws.total);
  if (!p) return TN_ENOMEM;
  int rc = batch_bind(b, p, b->ws.total);
  if (rc != TN_OK) {
    dev_free(p);
    b->d_ws = nullptr;
    return rc;
  }
  b->ws_owned = true;
  return TN_OK;
}

// One pass. ws: the workspace to run in; NULL for the batch's bound one
// (bound from the allocator when missing). A given ws holds the tables
// already; every launch then goes on st (no side streams, no timing events).
static int run_batch(tn_batch *b, char *ws, bool grad, const double *params, int n_sets, double *out, double *obj,
                     double *gobj, double *gnet_out, hipStream_t st) {
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
                  " needs more than 2^40 elements of adjoint working memory per parameter vector");
        return TN_ENOMEM;
      }
  const bool own_ws = ws != nullptr;
  if (!own_ws) {
    if (b->capturing) {
      if (!b->d_ws || b->items_dirty) {
        set_error("batch run under capture before its workspace and items are on the device");
        return TN_ESTATE;
      }
    } else {
      int rc = ensure_bound(b);
      if (rc != TN_OK) return rc;
    }
    ws = b->d_ws;
  }
  if (!b->level.empty() && !b->capturing) {
    int rc = task_grid(b);
    if (rc != TN_OK) return rc;
  }
  const int v = grad ? 1 : 0;
  FusedArgs a{};
  a.nets = wsp<DNet>(ws, b, grad ? WsLayout::NETS_GRAD : WsLayout::NETS_FWD);
  a.ops = wsp<DOp>(ws, b, WsLayout::OPS);
  a.recs = wsp<int4>(ws, b, WsLayout::RECS);
  a.tabs = wsp<int32_t>(ws, b, WsLayout::TABS);
  a.consts = wsp<void>(ws, b, WsLayout::CONSTS);
  a.ptens = wsp<DParam>(ws, b, WsLayout::PTENS);
  a.bound = wsp<void>(ws, b, WsLayout::BOUND);
  a.dbound = wsp<void>(ws, b, WsLayout::DBOUND);
  a.per_set = b->hp.per_set;
  a.task_net = wsp<int32_t>(ws, b, WsLayout::TASK_NET);
  // network-major output; the internal buffer is used when no pointer is given
  a.out_val = out ? out : wsp<double>(ws, b, WsLayout::VAL);
  a.out_grad = gnet_out ? gnet_out : wsp<double>(ws, b, WsLayout::GNET);
  a.n_params = b->n_params;
  a.n_sets = n_sets;
  a.n_tasks = (int)b->task_net.size() * n_sets;
  a.scratch_off = b->scratch_off[v];
  a.scal_off = b->scal_off[v];
  a.gacc_off = b->gacc_off[v];
  a.red_off = b->red_off[v];
  a.gbar_off = b->gbar_off[v];
  hipError_t e = launch_bind(b->dtype, wsp<DParam>(ws, b, WsLayout::SLOTS), (int)b->hp.slots.size(), params, b->n_params,
                             n_sets, b->hp.per_set, wsp<void>(ws, b, WsLayout::BOUND), grad ? wsp<void>(ws, b, WsLayout::DBOUND) : nullptr, st);
  if (e != hipSuccess) {
    b->poisoned = true;
    return hip_fail(e, "binding launch");
  }
  // streams of the global-arena (sg) and level (sl) executors: forked when
  // two or more executors have work
  hipStream_t sg = st, sl = st;
  const bool fork = b->ev_fork != nullptr && !own_ws;
  if (fork) {
    e = hipEventRecord(he(b->ev_fork), st);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      if (b->side[i]) e = hipStreamWaitEvent(hs(b->side[i]), he(b->ev_fork), 0);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "stream fork");
    }
    if (b->side[0]) sg = hs(b->side[0]);
    if (b->side[1]) sl = hs(b->side[1]);
  }
  // the level executor first: its task executor fills the chip, the fused
  // launches fill in around it
  if (!b->level.empty()) {
    const int prec = b->dtype == TN_C128 ? TN_MFMA_FP64 : b->mfma_prec;
    LvlArgs la{};
    la.n_sets = n_sets;
    la.max_sets = b->max_sets;
    la.ctrl = wsp<int32_t>(ws, b, WsLayout::CTRL);
    la.trecs = wsp<int4>(ws, b, WsLayout::TRECS);
    la.arena = wsp<void>(ws, b, WsLayout::LARENA);
    la.split = wsp<void>(ws, b, WsLayout::LSPLIT);
    la.scal = wsp<double>(ws, b, WsLayout::LSCAL);
    la.part = wsp<double>(ws, b, WsLayout::LPART);
    la.tabs = a.tabs;
    la.consts = a.consts;
    la.ptens = a.ptens;
    la.bound = a.bound;
    la.dbound = a.dbound;
    la.per_set = b->hp.per_set;
    la.n_sets_total = n_sets;
    la.n_params = b->n_params;
    la.with_grad = grad ? 1 : 0;
    la.out_val = a.out_val;
    la.out_grad = a.out_grad;
    for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
      const LevelGroup &g = b->groups[gi];
      la.set0 = 0;
      if (g.tasked) {
        la.items = wsp<PItem>(ws, b, v ? WsLayout::TITEMS1 : WsLayout::TITEMS0);
        la.tnets = wsp<TNet>(ws, b, v ? WsLayout::TNETS1 : WsLayout::TNETS0) + g.tnet0;
        la.n_tnets = (int)g.lv.size();
        e = task_reset(la, sl);
        if (e != hipSuccess) break;
        TimedLaunch tl = timing_begin(b, 1, own_ws, sl);
        e = task_run(prec, la, b->task_grid, sl);
        timing_end(b, 1, sl, e, tl);
      } else {
        TimedLaunch tl = timing_begin(b, 1, own_ws, sl);
        for (int i = g.item0[v]; i < g.item0[v] + g.n_items[v] && e == hipSuccess; ++i)
          e = item_launch(prec, b->items[v][i], la, sl);
        timing_end(b, 1, sl, e, tl);
      }
    }
    for (size_t q = 0; q < b->lsolo.size() && e == hipSuccess; ++q) {
      const LevelNet &ln = b->level[b->lsolo[q]];
      for (int s0 = 0; s0 < n_sets && e == hipSuccess; s0 += ln.chunk) {
        la.set0 = s0;
        la.n_sets = std::min(ln.chunk, n_sets - s0);
        for (int i = b->solo_begin[v][q]; i < b->solo_begin[v][q + 1] && e == hipSuccess; ++i)
          e = item_launch(prec, b->solo_items[v][i], la, sl);
      }
    }
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "level executor launch");
    }
  }
  if (a.n_tasks > 0) {
    const int spw = b->spw[v];
    if (spw > 1) {
      a.recs = wsp<int4>(ws, b, spw == 4 ? WsLayout::SRECS0 : WsLayout::SRECS1);
      a.set_stride = b->set_stride[v];
      a.max_comp = std::max(1, b->hp.max_comp);
      a.n_groups = (n_sets + spw - 1) / spw;
      a.n_tasks = (int)b->task_net.size() * a.n_groups;
    }
    // resident workgroups, balanced so every one runs the same number of tasks
    const int cap = std::max(1, std::min(grad ? b->grid_grad : b->grid_fwd, a.n_tasks));
    const int rounds = (a.n_tasks + cap - 1) / cap;
    const int grid = (a.n_tasks + rounds - 1) / rounds;
    a.per_block = rounds;
    TimedLaunch tl = timing_begin(b, 0, own_ws, st);
    if (spw > 1)
      e = launch_fused_sets(b->dtype, grad, spw, a, grid, grad ? b->lds_grad : b->lds_fwd, st);
    else
      e = launch_fused(b->dtype, b->block, grad, rec_only(b, v), false, a, grid, grad ? b->lds_grad : b->lds_fwd, st);
    timing_end(b, 0, st, e, tl);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "fused executor launch");
    }
  }
  if (!b->gtask_net.empty()) {
    const tn_batch::GLayout &gl = b->gl[v];
    FusedArgs g = a;
    g.recs = wsp<int4>(ws, b, WsLayout::RECS);
    g.task_net = wsp<int32_t>(ws, b, WsLayout::GTASK_NET);
    g.n_tasks = (int)b->gtask_net.size() * n_sets;
    g.scratch_off = gl.scratch_off;
    g.scal_off = gl.scal_off;
    g.gacc_off = gl.gacc_off;
    g.red_off = gl.red_off;
    g.garena = wsp<void>(ws, b, WsLayout::GARENA);
    g.garena_stride = b->gstride;
    const int cap = std::max(1, std::min(std::min(gl.grid, b->gslots), g.n_tasks));
    const int rounds = (g.n_tasks + cap - 1) / cap;
    g.per_block = rounds;
    TimedLaunch tl = timing_begin(b, 2, own_ws, sg);
    e = launch_fused(b->dtype, 256, grad, false, true, g, (g.n_tasks + rounds - 1) / rounds, gl.lds, sg);
    timing_end(b, 2, sg, e, tl);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "global-arena executor launch");
    }
  }
  if (fork) {
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      if (!b->side[i]) continue;
      e = hipEventRecord(he(b->ev_join[i]), hs(b->side[i]));
      if (e == hipSuccess) e = hipStreamWaitEvent(st, he(b->ev_join[i]), 0);
    }
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "stream join");
    }
  }
  if (obj || (grad && gobj)) {
    e = launch_combine(a.out_val, a.out_grad, wsp<double>(ws, b, WsLayout::COEF), b->offset, b->n_nets, n_sets,
                       b->n_params, obj, grad ? gobj : nullptr, st);
    if (e != hipSuccess) {
      b->poisoned = true;
      return hip_fail(e, "combine launch");
    }
  }
  return TN_OK;
}

int batch_contract(tn_batch *b, const double *params, int n_sets, double *out, double *obj, void *stream) {
  return run_batch(b, nullptr, false, params, n_sets, out, obj, nullptr, nullptr, (hipStream_t)stream);
}

int batch_grad(tn_batch *b, const double *params, int n_sets, double *out, double *obj, double *grad, double *gnet,
               void *stream) {
  return run_batch(b, nullptr, true, params, n_sets, out, obj, grad, gnet, (hipStream_t)stream);
}

// --- allocation-free runs ----------------------------------------------------------------------
// For callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation): a batch whose workspace
// fits runs in this fixed array instead of a bound workspace. Each device
// holds its own copy until the process ends. Host code reaches it only
// through the address hipGetSymbolAddress gives on that device (the array's
// name is a host-side stand-in there). Every call on a device shares the
// array: each call copies the batch's program arrays in again, and calls
// that overlap on one device race.
constexpr int64_t kStaticScratchBytes = int64_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static char *g_scratch[kMaxDevices];  // per device: the array's device address, once looked up

static int scratch_base(char **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("tn_batch_grad_noalloc: device ordinal beyond " + std::to_string(kMaxDevices));
    return TN_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      set_error("hipGetSymbolAddress(scratch): no address");
      return TN_EDEVICE;
    }
    g_scratch[dev] = static_cast<char *>(p);
  }
  *out = g_scratch[dev];
  return TN_OK;
}

int batch_grad_noalloc(tn_batch *b, const double *params, int n_sets, double *out, double *obj, double *grad,
                       double *gnet, void *stream) {
  if (b->ws.total > kStaticScratchBytes) {
    set_error("tn_batch_grad_noalloc: the batch needs " + std::to_string(b->ws.total) +
              " bytes of workspace; the static scratch holds " + std::to_string(kStaticScratchBytes));
    return TN_EINVAL;
  }
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  if ((!params && b->n_params > 0) || n_sets < 1 || n_sets > b->max_sets) {
    set_error("batch run: n_sets out of range or params NULL");
    return TN_EINVAL;
  }
  char *ws = nullptr;
  int rc = scratch_base(&ws);
  if (rc != TN_OK) return rc;
  const hipStream_t st = (hipStream_t)stream;
  // launch shapes from the device's occupancy (queries only)
  if ((rc = layout_lds(b, 0)) != TN_OK || (rc = layout_lds(b, 1)) != TN_OK || (rc = layout_gmem(b)) != TN_OK) return rc;
  if ((rc = upload_tables(b, ws, st, true, true)) != TN_OK) {
    b->poisoned = rc == TN_EDEVICE;
    return rc;
  }
  return run_batch(b, ws, true, params, n_sets, out, obj, grad, gnet, st);
}

int batch_run_graph(tn_batch *b, int with_grad, const double *params, int n_sets, double *out, double *obj,
                    double *grad, double *grad_net, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!st) {
    set_error("tn_batch_run_graph: needs a non-default stream (graph capture)");
    return TN_EINVAL;
  }
  if (b->poisoned) {
    set_error("batch poisoned by an earlier device error");
    return TN_ESTATE;
  }
  int rc = ensure_bound(b);  // uploads happen outside the capture
  if (rc != TN_OK) return rc;
  if (!b->level.empty() && (rc = task_grid(b)) != TN_OK) return rc;
  tn_batch::GraphCache &g = b->gc;
  const bool hit = g.exec && g.with_grad == with_grad && g.n_sets == n_sets && g.params == params && g.out == out &&
                   g.obj == obj && g.grad == grad && g.grad_net == grad_net && g.stream == (void *)st;
  if (!hit) {
    graph_clear(b);
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    b->capturing = true;
    rc = run_batch(b, nullptr, with_grad != 0, params, n_sets, out, obj, grad, with_grad ? grad_net : nullptr, st);
    b->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != TN_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    g.graph = graph;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    g.exec = exec;
    g.with_grad = with_grad;
    g.n_sets = n_sets;
    g.params = params;
    g.out = out;
    g.obj = obj;
    g.grad = grad;
    g.grad_net = grad_net;
    g.stream = st;
  }
  hipError_t e = hipGraphLaunch((hipGraphExec_t)g.exec, st);
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
  int rc = ensure_bound(b);
  if (rc != TN_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  reps = std::max(1, reps);
  std::map<std::string, int> found;
  graph_clear(b);
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
      float ms = time_ms(st, reps, [&] { return run_batch(b, nullptr, true, params, n_sets, nullptr, nullptr, nullptr, nullptr, st); },
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
      float ms = time_ms(st, reps, [&] { return run_batch(b, nullptr, false, params, n_sets, nullptr, nullptr, nullptr, nullptr, st); },
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
  // (2) large level ops: per shape class, each tile shape of the matrix-core
  // item and the thin item, timed as an item of the pass's parameter-vector
  // count on scratch operands (item mode only: the task executor puts every
  // eligible product on the matrix cores, tiled by its widths)
  std::map<std::string, DOp> classes;
  std::vector<char> tasked(b->level.size(), 0);
  for (const LevelGroup &g : b->groups)
    if (g.tasked)
      for (int l : g.lv) tasked[l] = 1;
  for (size_t l = 0; l < b->level.size(); ++l)
    for (int v = 0; v < 2; ++v) {
      if (tasked[l]) continue;
      const LevelNet &ln = b->level[l];
      for (int o = 0; o < ln.n_ops[v]; ++o) {
        const DOp &op = b->hp.ops[ln.op_begin[v] + o];
        if (mfma_eligible(b->dtype, op)) classes.emplace(shape_class(b->dtype, op, b->mfma_prec), op);
      }
    }
  const int eb = b->dtype == TN_C128 ? 16 : 8;
  const int prec = b->dtype == TN_C128 ? TN_MFMA_FP64 : b->mfma_prec;
  for (auto &kv : classes) {
    DOp op = kv.second;
    const int64_t nx = (int64_t)1 << (op.nFX + op.nS), ny = (int64_t)1 << (op.nS + op.nFY);
    const int64_t nz = (int64_t)1 << (op.nFX + op.nFY);
    // as many parameter vectors as the pass has, within 2^28 elements of scratch
    const int sets_t = (int)std::max<int64_t>(1, std::min<int64_t>(n_sets, ((int64_t)1 << 28) / (nx + ny + nz)));
    void *buf = dev_alloc((size_t)(nx + ny + nz) * sets_t * eb);
    if (!buf) continue;  // no room to tune this class: keep the default
    HIPCHK(hipMemset(buf, 0, (size_t)(nx + ny + nz) * sets_t * eb));
    op.x = 0;
    op.y = (int32_t)nx;
    op.z = (int32_t)(nx + ny);
    LevelNet ln;  // a one-op program on the scratch
    ln.n_ops[0] = 1;
    ln.stride[0] = nx + ny + nz;
    ItemCtx c = item_ctx(b);
    std::vector<DOp> one{op};
    c.ops = &one;
    c.split_target = 0;
    std::vector<PItem> ti;
    int64_t sn = 0, pn = 0;
    c.all_thin = true;
    network_items(c, ln, 0, sets_t, 0, 0, 0, 0, false, ti, &sn, &pn);
    c.all_thin = false;
    LvlArgs la{};
    la.arena = buf;
    la.n_sets = sets_t;
    la.tabs = ws_ptr<int32_t>(b, WsLayout::TABS);
    int rcl = TN_OK;
    // candidates: the tile shapes (complex128: 64 x 64 only), then the thin
    // item; item 1 of each list is the op (item 0 sets up, the last writes
    // outputs)
    int best_v = 1;
    float best_t = 1e30f;
    std::map<std::string, int> force;
    c.use_mfma = &force;
    for (int v : b->dtype == TN_C128 ? std::vector<int>{2} : std::vector<int>{2, 3, 4}) {
      force[kv.first] = v;
      std::vector<PItem> mi;
      network_items(c, ln, 0, sets_t, 0, 0, 0, 0, false, mi, &sn, &pn);
      const float t = time_ms(st, reps, [&] { return item_launch(prec, mi[1], la, st) == hipSuccess ? TN_OK : TN_EDEVICE; }, rcl);
      if (rcl != TN_OK) break;
      found["time_ns_tile" + std::to_string(v - 1) + ":" + kv.first + ":sets" + std::to_string(sets_t)] =
          (int)std::min(2e9f, t * 1e6f);
      if (t < best_t) {
        best_t = t;
        best_v = v;
      }
    }
    // the thin kernel is not a candidate for large products (2^24 and more
    // complex multiply-adds per parameter vector): the matrix cores win there
    float t_thin = 1e30f;
    if (rcl == TN_OK && op.nFX + op.nS + op.nFY < 24)
      t_thin = time_ms(st, reps, [&] { return item_launch(prec, ti[1], la, st) == hipSuccess ? TN_OK : TN_EDEVICE; }, rcl);
    (void)hipStreamSynchronize(st);
    dev_free(buf);
    if (rcl != TN_OK) {
      b->poisoned = true;
      set_error("tn_batch_autotune: launch failed");
      return TN_EDEVICE;
    }
    b->use_mfma[kv.first] = best_t <= t_thin ? best_v : 0;
    found["mfma:" + kv.first] = b->use_mfma[kv.first];
    // measured times (ns, at sets_t angle sets), recorded for inspection only
    if (t_thin < 1e29f)
      found["time_ns_thin:" + kv.first + ":sets" + std::to_string(sets_t)] = (int)std::min(2e9f, t_thin * 1e6f);
  }
  write_cache(cache_path, found);
  return plan_level(b);
}

int batch_kernel_timing(tn_batch *b, int enable) {
  b->timing = enable != 0;
  if (!b->timing) drop_timing_events(b);
  return TN_OK;
}

int batch_kernel_time(tn_batch *b, int kind, int *n, double *total_ms) {
  if (kind < 0 || kind > 2) {
    set_error("tn_batch_kernel_time: executor must be TN_EXEC_FUSED, TN_EXEC_LEVEL or TN_EXEC_GLOBAL");
    return TN_EINVAL;
  }
  double sum = 0.0;
  int cnt = 0;
  hipError_t e = hipSuccess;
  for (auto &pr : b->tev[kind]) {
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(he(pr.second));
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, he(pr.first), he(pr.second));
    if (e == hipSuccess) {
      sum += ms;
      ++cnt;
    }
  }
  for (auto &pr : b->tev[kind]) {
    (void)hipEventDestroy(he(pr.first));
    (void)hipEventDestroy(he(pr.second));
  }
  b->tev[kind].clear();
  if (e != hipSuccess) return hip_fail(e, "tn_batch_kernel_time");
  *n = cnt;
  *total_ms = sum;
  return TN_OK;
}

int batch_set_precision(tn_batch *b, int prec) {
  graph_clear(b);
  return plan_set_precision(b, prec);
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
    if (b->uploaded) {
      int rc;
      if ((rc = layout_lds(b, 0)) != TN_OK || (rc = layout_lds(b, 1)) != TN_OK) return rc;
    }
  }
  for (auto &kv : m)
    if (kv.first.rfind("mfma:", 0) == 0 && kv.second >= 0 && kv.second <= 4) b->use_mfma[kv.first.substr(5)] = kv.second;
  graph_clear(b);
  return plan_level(b);
}

int stream_sync(void *stream) {
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  return TN_OK;
}

void batch_free(tn_batch *b) {
  if (!b) return;
  free_device(b);
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
  DParam *d_dp = static_cast<DParam *>(dev_alloc(dp.size() * sizeof(DParam)));
  if (!d_dp) return TN_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(d_dp, dp.data(), dp.size() * sizeof(DParam), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_bind(net.dtype, d_dp, (int)dp.size(), params, net.n_params, n_sets, (int)total, dst, nullptr, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dev_free(d_dp);
  if (e != hipSuccess) return hip_fail(e, "tn_bind_params");
  return TN_OK;
}

}  // namespace qtn
