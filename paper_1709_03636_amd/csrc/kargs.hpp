// Kernel arguments of the executors (device code and the runtime that
// launches it).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace qtn {

struct FusedArgs {
  const DNet *nets;
  const DOp *ops;
  const int4 *recs;
  const int32_t *tabs;
  const void *consts;
  const DParam *ptens;
  const void *bound;        // [set][per_set] parametric tensors (binding kernel output)
  const void *dbound;       // [set][per_set] their angle derivatives (adjoint programs)
  const int32_t *task_net;  // queue position -> network index (cost order)
  double *out_val;          // [net][set][2]
  double *out_grad;         // [net][set][n_params] (adjoint programs)
  int n_params, n_sets, n_tasks, per_set;
  int set_stride, n_groups, max_comp;  // set-packed executor: LDS elements per set, set groups, scalars per set
  int per_block;            // workgroup b runs tasks [b*per_block, (b+1)*per_block)
  void *garena;             // global-arena executor: workgroup b works in garena + b * garena_stride
  int64_t garena_stride;    // (elements)
  int scratch_off, scal_off, gacc_off, red_off, gbar_off;  // LDS byte offsets
};

// Arguments of the level executor: the buffers the items address (item
// kernels read the item from their own argument), and for the task executor
// its items, networks and task counter ctrl[0].
struct LvlArgs {
  const PItem *items;
  const TNet *tnets;
  const int4 *trecs;   // task executor: lane records of PK_TREC items (64 per record)
  int n_tnets;         // tasks = n_tnets * max_sets (network, parameter vector) pairs
  int max_sets;
  int32_t *ctrl;
  int n_sets;          // parameter vectors of this pass (tasks of later vectors return at once)
  int set0;            // first parameter vector of this pass (networks run in chunks of vectors)
  void *arena;         // level arena
  void *split;         // partial tiles of split matrix-core products
  double *scal;        // component scalars
  double *part;        // partial sums of rank-0 contractions
  const int32_t *tabs;
  const void *consts;  // constant leaf values (complex, the batch's dtype)
  const DParam *ptens; // parametric leaves of the level networks
  const void *bound;   // [set][per_set] bound parametric tensors
  const void *dbound;  // their angle derivatives
  int per_set;
  int n_sets_total;    // parameter vectors of the whole call (output row stride)
  int n_params;
  int with_grad;
  double *out_val;     // [net][set][2]
  double *out_grad;    // [net][set][n_params]
};

}  // namespace qtn
