// Level executor kernels: one item per launch (item mode: networks run one
// op at a time on the whole chip; the autotuner's trials), and the task
// executor, one persistent launch in which every workgroup runs whole
// (network, parameter vector) programs.
//
// Task executor: a workgroup takes the next task from a counter, then runs
// the network's items (built for one parameter vector) one after another on
// that vector's slice of the network's region, a barrier between items.
// Tasks share no memory, so no ordering between workgroups is needed (on
// this chip that ordering would cost an L2 write-back and invalidation per
// task). The tasks are numbered network-major with the networks in
// decreasing cost, so the longest finish first.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"
#include "kargs.hpp"
#include "lrec.hpp"
#include "task.hpp"

namespace qtn {

// Waves per SIMD the kernels are compiled for. Item kernels: the split-BF16
// 64 x 64 tile holds 132 registers unconstrained (3 waves per SIMD); capped
// at 128 it runs 4 without spills; the others keep the compiler's choice
// (FP64 would spill). Task executor: three workgroups per CU share its LDS
// (tile staging plus the small-tensor arena), so complex64 programs are
// built for 3 waves per SIMD (at most 168 registers).
template <int PREC>
constexpr int kMinWaves = PREC == TN_MFMA_BF16X3 ? 4 : 1;
template <int PREC>
constexpr int kTaskWaves = PREC == TN_MFMA_FP64 ? 1 : 3;
// LDS of a workgroup: the largest tile, and at least the 72 doubles of the
// FP64 sums; the item kernel double-buffers split-BF16 tiles.
template <int PREC>
constexpr int kItemLds = kTileLds<PREC> > 576 ? kTileLds<PREC> : 576;
template <int PREC>
constexpr int kItemKernelLds = PREC == TN_MFMA_BF16X3 ? 2 * kItemLds<PREC> : kItemLds<PREC>;

template <int PREC>
__global__ __launch_bounds__(256, kMinWaves<PREC>) void item_kernel(PItem it, LvlArgs a) {
  __shared__ __align__(16) char lds[kItemKernelLds<PREC>];
  run_item<PREC, false>(lds, nullptr, it, (int)blockIdx.x, (int)gridDim.x, a);
}

// The loop's only per-thread branch (thread 0 takes the next task) sits at
// its top, before the barrier that publishes the task, and every value the
// loop branches on is read into scalar registers: a thread-0 branch next to
// the back edge can be compiled into an inner loop that the other threads
// re-enter without thread 0.
//
// Item descriptors are staged through LDS: the next item's words are
// loaded (one word per thread, all at once) while the current item runs and
// stored before the barrier that ends it, so an item starts without a
// memory round trip per descriptor field. Every thread takes part (indices
// clamped; threads past the descriptor rewrite its padding word), keeping
// the loop free of per-thread branches.
// A PK_TREC item: a run of steps, wave w running the w-th of a step's small
// independent contractions (or leaf adjoint additions) from its lane record
// (the first step's loaded while the item before it ran, each later one
// while the step before it runs); the operands are in the LDS arena.
template <typename V>
__device__ __forceinline__ void run_rec(const V *xm, const V *ym, V *zm, const int4 &rec) {
  const uint32_t hdr = (uint32_t)__builtin_amdgcn_readfirstlane(rec.w);
  const uint32_t type = hdr & 7u;
  if (type == kRecLite) {
    switch ((hdr >> 3) & 15u) {
      case 0: contract_lite<V, 0>(xm, ym, zm, rec, hdr); break;
      case 1: contract_lite<V, 1>(xm, ym, zm, rec, hdr); break;
      default: contract_lite<V, 2>(xm, ym, zm, rec, hdr); break;
    }
  } else if (type == kRecWide) {
    contract_wide<V>(xm, ym, zm, rec, hdr);
  } else if (type == kRecNarrow) {
    contract_narrow<V>(xm, ym, zm, rec, hdr);
  } else if (type == kRecAcc) {
    acc_rec<V>(xm, zm, rec, hdr);
  }
}



constexpr int kItemWords = (int)(sizeof(PItem) / 4);
constexpr int kItemRow = (kItemWords + 4 + 3) & ~3;  // 16-byte rows with padding
static_assert(sizeof(PItem) % 4 == 0, "item descriptors are copied in whole words");

template <int PREC>
__global__ __launch_bounds__(256, kTaskWaves<PREC>) void task_kernel(LvlArgs a) {
  // the program's small tensors (arena), then the tile staging, which holds
  // small tensors too between the items that use it
  __shared__ __align__(16) char lsm[kLdsArenaBytes<PREC> + kItemLds<PREC>];
  char *const lar = lsm, *const lds = lsm + kLdsArenaBytes<PREC>;
  __shared__ __align__(16) int32_t s_item[2][kItemRow];  // current and next item descriptor
  __shared__ int s_task;
  constexpr int eb = PREC == TN_MFMA_FP64 ? 16 : 8;
  using V = typename std::conditional<PREC == TN_MFMA_FP64, double2, float2>::type;
  const int total = a.n_tnets * a.max_sets;
  const int word = min((int)threadIdx.x, kItemWords - 1), slot = min((int)threadIdx.x, kItemRow - 1);
  for (;;) {
    if (threadIdx.x == 0) s_task = __hip_atomic_fetch_add(a.ctrl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= total) return;  // uniform
    const int j = t / a.max_sets, s = t - j * a.max_sets;
    if (s < a.n_sets) {
      const TNet &tn = a.tnets[j];
      LvlArgs v = a;
      v.arena = (char *)a.arena + (tn.abase + (int64_t)s * tn.stride) * eb;
      v.scal = a.scal + tn.sbase + (int64_t)s * tn.n_comp * 2;
      v.set0 = s;
      v.n_sets = 1;
      v.n_sets_total = a.n_sets;
      const int i0 = __builtin_amdgcn_readfirstlane(tn.item0), n = __builtin_amdgcn_readfirstlane(tn.n_items);
      const int32_t *src = reinterpret_cast<const int32_t *>(a.items + i0);
      if (n > 0) s_item[0][slot] = src[word];
      __syncthreads();
      int4 rcur = make_int4(0, 0, 0, 0);  // this wave's lane record of the item (PK_TREC), loaded during the last one
      const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
      for (int i = 0; i < n; ++i) {
        const bool more = i + 1 < n;  // uniform
        int32_t next = 0;
        if (more) next = src[(int64_t)(i + 1) * kItemWords + word];
        const PItem &it = *reinterpret_cast<const PItem *>(s_item[i & 1]);
        // wave w loads the w-th lane record of the next item
        const int nr = __builtin_amdgcn_readfirstlane(it.nrec), nn = __builtin_amdgcn_readfirstlane(it.nrec_n);
        int4 rnext = make_int4(0, 0, 0, 0);
        if (wave < nn) rnext = a.trecs[(int64_t)(nr + wave) * kRecLanes + (threadIdx.x & (kRecLanes - 1))];
        const int kind = __builtin_amdgcn_readfirstlane(it.kind);
        if (kind == PK_TREC) {
          V *m = reinterpret_cast<V *>(lar);
          const int steps = __builtin_amdgcn_readfirstlane(it.lgl);
          const int32_t pk[6] = {__builtin_amdgcn_readfirstlane(it.a0), __builtin_amdgcn_readfirstlane(it.a1),
                                 __builtin_amdgcn_readfirstlane(it.a2), __builtin_amdgcn_readfirstlane(it.a3),
                                 __builtin_amdgcn_readfirstlane(it.a4), __builtin_amdgcn_readfirstlane(it.a5)};
          auto count = [&](int t) { return ((pk[t >> 4] >> (2 * (t & 15))) & 3) + 1; };
          int r = __builtin_amdgcn_readfirstlane(it.rec);
          int4 cur = rcur;
          for (int t = 0; t < steps; ++t) {
            const int c = count(t), cn = t + 1 < steps ? count(t + 1) : 0;
            // the next step's record of this wave is loaded while this step runs
            int4 nx = make_int4(0, 0, 0, 0);
            if (wave < cn) nx = a.trecs[(int64_t)(r + c + wave) * kRecLanes + (threadIdx.x & (kRecLanes - 1))];
            if (wave < c) run_rec<V>(m, m, m, cur);
            // steps on wave 0 alone follow each other without a barrier (a
            // wave's LDS accesses complete in order)
            if (cn > 0 && (c > 1 || cn > 1)) __syncthreads();
            cur = nx;
            r += c;
          }
        } else {
          const int cnt = __builtin_amdgcn_readfirstlane(kind == PK_MFMA ? it.count : 1);
          for (int r = 0; r < cnt; ++r) run_item<PREC, true>(lds, lar, it, r, cnt, v);
        }
        if (more) s_item[(i + 1) & 1][slot] = next;
        __syncthreads();  // the next item reads what this one wrote (same workgroup) and its descriptor
        rcur = rnext;
      }
    }
    __syncthreads();  // every thread has read s_task before it is rewritten
  }
}

__global__ __launch_bounds__(64) void task_reset_kernel(int32_t *ctrl) {
  if (threadIdx.x == 0) ctrl[0] = 0;
}

// --- host launchers ------------------------------------------------------------------------

const void *item_kernel_ptr(int prec) {
  switch (prec) {
    case TN_MFMA_BF16X3: return (const void *)item_kernel<TN_MFMA_BF16X3>;
    case TN_MFMA_FP64: return (const void *)item_kernel<TN_MFMA_FP64>;
    default: return (const void *)item_kernel<TN_MFMA_FP32>;
  }
}

const void *task_kernel_ptr(int prec) {
  switch (prec) {
    case TN_MFMA_BF16X3: return (const void *)task_kernel<TN_MFMA_BF16X3>;
    case TN_MFMA_FP64: return (const void *)task_kernel<TN_MFMA_FP64>;
    default: return (const void *)task_kernel<TN_MFMA_FP32>;
  }
}

// One item on it.count workgroups; prec: the batch's matrix-core precision
// (its dtype's kernel: TN_MFMA_FP64 for complex128).
hipError_t item_launch(int prec, const PItem &it, const LvlArgs &a, hipStream_t st) {
  if (it.count < 1) return hipSuccess;
  void *args[] = {(void *)&it, (void *)&a};
  return hipLaunchKernel(item_kernel_ptr(prec), dim3(it.count), dim3(256), args, 0, st);
}

// The task counter cleared (a kernel, so that captured graphs hold no
// memset node).
hipError_t task_reset(const LvlArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(task_reset_kernel, dim3(1), dim3(64), 0, st, a.ctrl);
  return hipGetLastError();
}

// The task executor on `grid` workgroups (after task_reset on the same stream).
hipError_t task_run(int prec, const LvlArgs &a, int grid, hipStream_t st) {
  void *args[] = {(void *)&a};
  return hipLaunchKernel(task_kernel_ptr(prec), dim3(grid), dim3(256), args, 0, st);
}

}  // namespace qtn
