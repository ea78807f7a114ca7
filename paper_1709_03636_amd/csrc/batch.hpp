// Host-side state of a batch: many networks x many parameter vectors.
//
// Planning (bplan.cpp, plain C++, no GPU calls) turns the networks' compiled
// programs into the arrays the kernels read (program descriptors, lane
// records, offset tables, constants), assigns every network to an executor
// (fused in LDS, fused on global-arena slots, or the level executor), lays
// out the level executor's items and task queue, and lays out the batch's
// device workspace. The runtime (runtime.hip) binds a workspace, uploads the
// arrays and launches. Device handles are kept as opaque pointers here.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace qtn {

constexpr int kLdsCap = 160 * 1024;
// Networks whose fused adjoint program needs more LDS than this run on the
// global-arena or level executor, so one large network does not lower the
// occupancy of all (the fused launch takes the largest program's LDS).
// Measured on the p=2 batches of 64 angle sets against 48 and 24 KiB: 32
// KiB was fastest on all but the 5-regular n=100 diagonal one (4-regular
// n=70 dense 3.1 -> 2.7 ms and diagonal 2.3 -> 1.0 ms; 3-regular n=60
// 0.68 -> 0.55 ms; 5-regular n=100 diagonal 4.1 -> 5.0 ms).
constexpr int64_t kFusedLdsMax = 32 * 1024;
constexpr int64_t kFusedLdsMaxHi = 48 * 1024;  // kept for some batches (plan_batch): three workgroups per CU
// Level arena budget: the networks of one group share it (more networks per
// launch, fewer groups one after another); a network alone
// processes its parameter vectors in chunks that fit. 32 GiB of the 288 GB.
constexpr int64_t kLevelBudget = 32ll << 30;
constexpr int64_t kMaxArenaElems = int64_t(1) << 31;  // global-arena executor: 32-bit element offsets per slot
constexpr int64_t kMaxLevelElems = int64_t(1) << 40;  // level executor: elements of one set's region
// Global-arena fused executor: networks too large for LDS whose whole task
// (forward + adjoint program of one parameter vector) has at most this many
// complex multiply-adds, and no step above a sixteenth of it.
constexpr int64_t kGmemMaxMacs = int64_t(1) << 20;
constexpr int64_t kGmemBudget = 16ll << 30;  // bytes of arena slots
// Most tasks (workgroups) of one thin item.
constexpr int64_t kItemMaxTasks = 65536;
// Split summed index of matrix-core items: an item whose tiles over all
// parameter vectors number fewer than kSplitTarget (default; QTN_SPLIT_TARGET)
// is split into up to 64 ranges (at least 512 summed entries each) until it
// has about kSplitTarget tasks, its partial tiles taking at most
// kSplitItemBytes of the network's split scratch.
constexpr int64_t kSplitTarget = 1024;
constexpr int64_t kSplitItemBytes = int64_t(512) << 20;


// Layout of one network's buffers in executor memory: constant leaves,
// parametric leaves, then the arena of intermediates/adjoints for each
// program variant (0 = forward, 1 = forward + adjoint).
struct NetLayout {
  std::vector<int64_t> coff, poff;
  int64_t n_const = 0, leaf_region = 0, ptens_elems = 0;
  std::vector<int64_t> off[2];
  int64_t arena[2] = {0, 0};
};
NetLayout make_layout(const Net &net);

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
  int64_t leaf_region = 0;                      // constants and parametric tensors: region [0, leaf_region)
  int chunk = 1;                                // parameter vectors per pass
  bool grad_ok = true;                          // the adjoint arena is addressable (< 2^31 elements)
  double cost = 0;                              // flops of forward + adjoint, one parameter vector
};

// Level networks whose parameter vectors all fit in the arena at once run
// in groups (groups one after another, sharing the arena): each network of a
// group owns an arena region, a region of component scalars, of rank-0
// partial sums and of split partial tiles. A group with at least task_min
// (network, parameter vector) pairs runs on the task executor (one launch;
// one workgroup per pair runs the network's items built for one vector);
// smaller groups launch their networks' items one by one (item mode).
struct LevelGroup {
  std::vector<int> lv;                              // indices into tn_batch::level
  std::vector<int64_t> abase, sbase, pbase, zbase;  // elements, doubles, doubles, elements
  std::vector<int64_t> zsize;                       // split scratch elements of each network
  int item0[2] = {0, 0}, n_items[2] = {0, 0};       // item mode: into tn_batch::items[variant]
  bool tasked = false;
  int tnet0 = 0;                                    // task executor: into tn_batch::tnets[variant]
};
constexpr int kTaskMin = 512;  // (network, vector) pairs a group needs for the task executor
constexpr double kGmemJoinMacs = 6e6;  // global-arena work (per vector) that joins the task executor alone

// Workspace layout: byte offsets of every device array of the batch.
struct WsLayout {
  enum {
    NETS_FWD, NETS_GRAD, OPS, TABS, RECS, SRECS0, SRECS1, TASK_NET, GTASK_NET, CONSTS, PTENS, SLOTS, COEF, BOUND,
    DBOUND, VAL, GNET, GARENA, LARENA, LSCAL, LPART, LSPLIT, TITEMS0, TITEMS1, TNETS0, TNETS1, TRECS, CTRL, N
  };
  int64_t off[N] = {};
  int64_t size[N] = {};
  int64_t total = 0;
};

}  // namespace qtn

struct tn_batch {
  int dtype = 0, n_nets = 0, n_params = 0, max_sets = 0, block = 128;
  int spw[2] = {1, 1};                 // angle sets per wave of the fused executor (1, 2 or 4), forward / adjoint
  int64_t fused_budget = 0;            // LDS bytes a fused workgroup may use
  double offset = 0;
  std::vector<double> coef;
  qtn::HostProgram hp;
  std::vector<float> consts_f;         // complex64 batches: hp.consts in FP32, as uploaded
  std::vector<int32_t> task_net;       // fused networks, in cost order
  std::vector<int32_t> gtask_net;      // networks on the global-arena fused executor, in cost order
  struct GLayout { int lds = 0, grid = 0, scratch_off = 0, scal_off = 0, gacc_off = 0, red_off = 0; } gl[2];
  int64_t gstride = 0;                 // elements per global-arena slot
  int gslots = 0;                      // slots (= most workgroups of one launch)
  // level executor
  std::vector<qtn::LevelNet> level;    // networks on the level executor
  std::vector<qtn::LevelGroup> groups; // level networks whose vectors all fit the arena at once
  std::vector<int> lsolo;              // level networks run one by one, in chunks of parameter vectors
  std::vector<qtn::PItem> items[2];    // item-mode items of the groups, per program variant (forward, adjoint)
  std::vector<qtn::PItem> titems[2];   // task-executor items (one parameter vector each)
  std::vector<qtn::TNet> tnets[2];     // task-executor networks, groups one after another
  std::vector<qtn::PItem> solo_items[2];  // items of the networks run alone (one launch each)
  std::vector<int> solo_begin[2];      // first solo item of each lsolo network, plus an end marker
  int64_t cap_titems[2] = {0, 0};      // workspace room for task-executor items
  std::vector<int32_t> trecs;          // task-executor lane records (both variants), 4 ints x 64 lanes each
  int64_t cap_trecs = 0;               // workspace room for them (ints)
  int task_min = qtn::kTaskMin;        // pairs a group needs for the task executor (QTN_TASK_MIN)
  int64_t larena_elems = 0, lscal_doubles = 0, lpart_doubles = 0, lsplit_elems = 0;
  int64_t split_target = 0;            // tasks a split matrix-core item aims at (0: no splits)
  std::map<std::string, int> use_mfma; // autotuner: shape class of a large op -> 0 thin, 1 matrix cores
                                       // (tile by widths), 2-4 matrix cores on 64 x 64 / 16 x 64 / 64 x 16 tiles
  int mfma_prec = TN_MFMA_FP32;        // matrix-core precision of large steps (complex128: TN_MFMA_FP64)
  double flops_fwd = 0, bytes_fwd = 0, flops_grad = 0, bytes_grad = 0;
  double exec_flops[3] = {0, 0, 0}, exec_bytes[3] = {0, 0, 0};  // per executor (fused, level, global), fwd + adjoint
  int64_t level_bytes = 0;
  qtn::WsLayout ws;
  // device state (runtime.hip)
  char *d_ws = nullptr;                // the workspace (caller's, or owned when ws_owned)
  bool ws_owned = false;
  bool uploaded = false;               // program arrays are in the workspace
  bool items_dirty = true;             // item lists changed since the last upload
  int lds_fwd = 0, lds_grad = 0, grid_fwd = 0, grid_grad = 0, task_grid = 0, task_grid_prec = 0;
  int scratch_off[2] = {0, 0}, scal_off[2] = {0, 0}, gacc_off[2] = {0, 0}, red_off[2] = {0, 0},
      gbar_off[2] = {0, 0}, set_stride[2] = {0, 0};
  bool poisoned = false;
  bool timing = false, capturing = false;
  // with work on two or more executors, the global-arena executor runs on
  // side[0] and the level executor on side[1], forked from the caller's
  // stream after binding and joined before the combine
  void *side[2] = {nullptr, nullptr};
  void *ev_fork = nullptr, *ev_join[2] = {nullptr, nullptr};
  std::vector<std::pair<void *, void *>> tev[3];  // timing event pairs per executor (fused, level, global)
  struct GraphCache {
    void *exec = nullptr, *graph = nullptr;
    int with_grad = -1, n_sets = -1;
    const void *params = nullptr, *out = nullptr, *obj = nullptr, *grad = nullptr, *grad_net = nullptr;
    void *stream = nullptr;
  } gc;
};

namespace qtn {

// What decides a level network's items: dtype, matrix-core precision and
// the autotuner's choices (use_mfma NULL: every eligible op on the matrix
// cores; all_thin: none).
struct ItemCtx {
  int dtype = 0, mfma_prec = 0;
  int64_t split_target = 0;
  const std::map<std::string, int> *use_mfma = nullptr;
  bool all_thin = false;
  int force_tile = -1;  // >= 0: every matrix-core op takes this tile shape (scratch sizing)
  bool one_wg = false;  // items for one workgroup and one vector (task executor): no split sums, one
                        // workgroup per rank-0 sum and set-up
  int lds_elems = 0;    // one_wg: elements of the workgroup's LDS arena for small tensors (0: none)
  int tile_elems = 0;   // one_wg: elements of the tile staging usable between the items that need it
  std::vector<int32_t> *trecs = nullptr;  // one_wg: lane records of PK_TREC items are appended here
  const std::vector<DOp> *ops = nullptr;
  const std::vector<int32_t> *tabs = nullptr;
};

// bplan.cpp
int plan_batch(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch *b);
// Level items and queues for the current matrix-core choices (precision,
// autotuner decisions); items_dirty is set.
int plan_level(tn_batch *b);
void plan_workspace(tn_batch *b);
std::string shape_class(int dtype, const DOp &op, int prec);
int level_prec(const tn_batch *b, const DOp &op);
int level_prec(const ItemCtx &c, const DOp &op);
ItemCtx item_ctx(const tn_batch *b);
bool mfma_eligible(int dtype, const DOp &op);
int level_tile(const ItemCtx &c, const DOp &op);
int mfma_tiles(const DOp &op, int shape);
int mfma_variant(const DOp &op, int prec, int shape);
// Items of one level network over n_sets parameter vectors (region offsets
// as given); appends to `out`.
void network_items(const ItemCtx &c, const LevelNet &ln, int v, int n_sets, int64_t abase, int64_t sbase,
                   int64_t pbase, int64_t zbase, bool allow_split, std::vector<PItem> &out, int64_t *split_need,
                   int64_t *part_need);
int batch_info(const tn_batch *b, tn_batch_stats *s);
int batch_create(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch **out);
int64_t batch_workspace_bytes(const tn_batch *b);
int plan_set_precision(tn_batch *b, int prec);
// LDS bytes of the fused executor's set-packed layout with S sets per wave
// (and the per-set stride and offsets), and whether it is available for a
// program variant within an LDS budget.
int set_lds_layout(const tn_batch *b, int S, int variant, int *stride, int *scal_off, int *gacc_off);
bool sets_fit(const tn_batch *b, int S, int64_t budget, int variant);

}  // namespace qtn
