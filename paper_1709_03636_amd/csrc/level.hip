// Level executor: runs network programs whose tensors do not fit in one
// workgroup's LDS. Every buffer of a (network, parameter vector) pair lives
// in a global-memory arena slice, with the same addressing as the fused
// executor (free-index deposit plus a per-op offset table for the summed
// index, eq. (1)). Networks stepped together run step k of all of them as
// one grouped launch per kind (thin contractions, leaf adjoints; matrix-core
// products in mfma.hip), over all parameter vectors at once; a network run
// alone takes one launch per op over a chunk of parameter vectors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "group.hpp"
#include "internal.hpp"
#include "thin.hpp"

namespace qtn {

// Z[set][c] = sum_k X[set][fx(c) + tx(k)] * Y[set][fy(c) + ty(k)]; one output per thread.
template <typename V>
__global__ __launch_bounds__(256) void level_contract_kernel(LevelArgs a, DOp op, DRuns ru,
                                                             const int32_t *__restrict__ tab,
                                                             const int32_t *__restrict__ tabB) {
  const int lgOut = op.nFX + op.nB + op.nFY;
  const int64_t nOut = (int64_t)1 << lgOut;
  const int64_t total = nOut * a.n_sets;
  V *arena = reinterpret_cast<V *>(a.arena);
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t set = g >> lgOut;
    const uint32_t c = (uint32_t)(g & (nOut - 1));
    V *base = arena + set * a.stride;
    base[op.z + c] = thin_output(base, op, ru, tab, tabB, c, 0, 1);
  }
}

// Rank-0 result, FP64: workgroup g of parameter vector s sums the summed
// entries g, g + G*256, ... into part[s][g]; a second kernel adds the G
// partial sums in index order (a fixed tree: results do not depend on
// scheduling).
template <typename V>
__global__ __launch_bounds__(256) void level_scalar_part_kernel(LevelArgs a, DOp op, const int32_t *__restrict__ tab,
                                                                double *__restrict__ part) {
  __shared__ double red[2][4];
  const int set = blockIdx.y;
  const int G = gridDim.x;
  const V *base = reinterpret_cast<const V *>(a.arena) + set * a.stride;
  const int64_t K = (int64_t)1 << op.nS;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < K; k += (int64_t)G * 256) {
    const int2 o = l_tab(tab, op.nS, (int)k);
    const double2 x = l_d2(base[op.x + o.x]);
    const double2 y = l_d2(base[op.y + o.y]);
    re += x.x * y.x - x.y * y.y;
    im += x.x * y.y + x.y * y.x;
  }
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = re;
    red[1][threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[((size_t)set * G + blockIdx.x) * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[((size_t)set * G + blockIdx.x) * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ void level_scalar_final_kernel(LevelArgs a, DOp op, const double *__restrict__ part, int G) {
  const int set = blockIdx.x * blockDim.x + threadIdx.x;
  if (set >= a.n_sets) return;
  double re = 0.0, im = 0.0;
  for (int g = 0; g < G; ++g) {
    re += part[((size_t)set * G + g) * 2];
    im += part[((size_t)set * G + g) * 2 + 1];
  }
  a.scal[((size_t)set * a.n_comp + op.z) * 2] = re;
  a.scal[((size_t)set * a.n_comp + op.z) * 2 + 1] = im;
}

// Adjoint seed of component aux0: product of the other component scalars.
template <typename V>
__global__ void level_seed_kernel(LevelArgs a, DOp op) {
  const int set = blockIdx.x * blockDim.x + threadIdx.x;
  if (set >= a.n_sets) return;
  double pr = 1.0, pi = 0.0;
  for (int j = 0; j < a.n_comp; ++j) {
    if (j == op.aux0) continue;
    const double sr = a.scal[((size_t)set * a.n_comp + j) * 2], si = a.scal[((size_t)set * a.n_comp + j) * 2 + 1];
    const double nr = pr * sr - pi * si, ni = pr * si + pi * sr;
    pr = nr;
    pi = ni;
  }
  V *base = reinterpret_cast<V *>(a.arena) + set * a.stride;
  base[op.z] = l_from<V>(make_double2(pr, pi));
}

// Leaf adjoint added into its tensor's canonical-layout accumulator at y.
template <typename V>
__global__ __launch_bounds__(256) void level_leafgrad_kernel(LevelArgs a, DOp op, const int32_t *__restrict__ tab) {
  const int n = 1 << op.nFX;
  const int64_t total = (int64_t)n * a.n_sets;
  V *arena = reinterpret_cast<V *>(a.arena);
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t set = g / n;
    const int i = (int)(g - set * n);
    V *base = arena + set * a.stride;
    V v = base[op.y + tab[i]];
    const V x = base[op.x + i];
    v.x += x.x;
    v.y += x.y;
    base[op.y + tab[i]] = v;
  }
}

// Set-up of a chunk: constants and bound parametric tensors into every
// slice, adjoint accumulators cleared. Entries of one slice: `n_copy`
// from consts, then per tensor from the bound-tensor buffer.
template <typename V>
__global__ __launch_bounds__(256) void level_setup_kernel(LevelArgs a, const V *__restrict__ consts, int n_const,
                                                          const DParam *__restrict__ pt, int n_pt,
                                                          const V *__restrict__ bound, int per_set, int set0,
                                                          int zero_begin, int zero_n) {
  const int set = blockIdx.y;
  V *base = reinterpret_cast<V *>(a.arena) + set * a.stride;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_const; e += gridDim.x * blockDim.x) base[e] = consts[e];
  const V *bs = bound + (size_t)(set0 + set) * per_set;
  for (int t = 0; t < n_pt; ++t) {
    const DParam d = pt[t];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (1 << d.bits); e += gridDim.x * blockDim.x)
      base[d.off + e] = bs[d.slot + e];
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < zero_n; e += gridDim.x * blockDim.x) {
    V z;
    z.x = 0;
    z.y = 0;
    base[zero_begin + e] = z;
  }
}

// Outputs of a chunk: value = product of component scalars; gradient =
// sum over parametric tensors of coeff * Re <Gbar, dG/dtheta> in FP64.
template <typename V>
__global__ __launch_bounds__(256) void level_finish_kernel(LevelArgs a, const DParam *__restrict__ pt, int n_pt,
                                                           const V *__restrict__ dbound, int per_set, int set0,
                                                           int net, int n_sets_total, int n_params,
                                                           double *__restrict__ out_val, double *__restrict__ out_grad,
                                                           int with_grad) {
  __shared__ double red[4];
  __shared__ double gacc[64];
  const int set = blockIdx.x;
  const V *base = reinterpret_cast<const V *>(a.arena) + set * a.stride;
  const int gs = set0 + set;
  if (threadIdx.x == 0) {
    double pr = 1.0, pi = 0.0;
    for (int j = 0; j < a.n_comp; ++j) {
      const double sr = a.scal[((size_t)set * a.n_comp + j) * 2], si = a.scal[((size_t)set * a.n_comp + j) * 2 + 1];
      const double nr = pr * sr - pi * si, ni = pr * si + pi * sr;
      pr = nr;
      pi = ni;
    }
    out_val[((size_t)net * n_sets_total + gs) * 2] = pr;
    out_val[((size_t)net * n_sets_total + gs) * 2 + 1] = pi;
  }
  if (!with_grad) return;
  for (int p0 = 0; p0 < n_params; p0 += 64) {
    for (int p = threadIdx.x; p < 64; p += blockDim.x) gacc[p] = 0.0;
    __syncthreads();
    const V *dset = dbound + (size_t)gs * per_set;
    for (int t = 0; t < n_pt; ++t) {
      const DParam d = pt[t];
      if (d.param < p0 || d.param >= p0 + 64) continue;
      double acc = 0.0;
      for (int e = threadIdx.x; e < (1 << d.bits); e += 256) {
        const double2 g = l_d2(base[d.goff + e]);
        const double2 dv = l_d2(dset[d.slot + e]);
        acc += g.x * dv.x - g.y * dv.y;
      }
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
      __syncthreads();
      if (threadIdx.x == 0) gacc[d.param - p0] += d.coeff * (red[0] + red[1] + red[2] + red[3]);
      __syncthreads();
    }
    for (int p = threadIdx.x; p < 64 && p0 + p < n_params; p += blockDim.x)
      out_grad[((size_t)net * n_sets_total + gs) * n_params + p0 + p] = gacc[p];
    __syncthreads();
  }
}

// --- grouped launches: one step of many networks ---------------------------------------------

// Thin contractions and leaf adjoints of several networks at once (one op of
// one network per item; thin_item).
template <typename V>
__global__ __launch_bounds__(256) void level_group_contract_kernel(const LItem *__restrict__ items,
                                                                   const int32_t *__restrict__ blk, int n, V *arena,
                                                                   int n_sets, const int32_t *__restrict__ tabs) {
  int rank, count;
  const LItem &it = items[group_item(blk, n, &rank, &count)];
  thin_item<V>(it, rank, count, arena, n_sets, tabs);
}

// --- host launchers ------------------------------------------------------------------------
bool mfma_eligible(int dtype, const DOp &op);
hipError_t mfma_contract(const LevelArgs &a, const DOp &op, const int32_t *tab, int prec, hipStream_t st);

static inline int grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

template <typename V>
static hipError_t level_op_t(const LevelArgs &a, const DOp &op, const int32_t *tabs, hipStream_t st) {
  const int32_t *tab = tabs + op.tab;
  switch (op.type) {
    case OP_CONTRACT: {
      int64_t total = ((int64_t)1 << (op.nFX + op.nB + op.nFY)) * a.n_sets;
      DRuns ru;
      pack_runs(op.maskX, ru.runsX);
      pack_runs(op.maskY, ru.runsY);
      hipLaunchKernelGGL(level_contract_kernel<V>, dim3(grid_for(total)), dim3(256), 0, st, a, op, ru, tab,
                         tabs + op.tabB);
      break;
    }
    case OP_SCALAR: {
      // about four summed entries per thread, at most kScalarParts workgroups per set
      const int64_t K = (int64_t)1 << op.nS;
      const int G = (int)std::min<int64_t>(kScalarParts, std::max<int64_t>(1, K / 1024));
      hipLaunchKernelGGL(level_scalar_part_kernel<V>, dim3(G, a.n_sets), dim3(256), 0, st, a, op, tab, a.part);
      hipLaunchKernelGGL(level_scalar_final_kernel, dim3((a.n_sets + 63) / 64), dim3(64), 0, st, a, op, a.part, G);
      break;
    }
    case OP_SEED:
      hipLaunchKernelGGL(level_seed_kernel<V>, dim3((a.n_sets + 63) / 64), dim3(64), 0, st, a, op);
      break;
    default: {
      int64_t total = ((int64_t)1 << op.nFX) * a.n_sets;
      hipLaunchKernelGGL(level_leafgrad_kernel<V>, dim3(grid_for(total)), dim3(256), 0, st, a, op, tab);
      break;
    }
  }
  return hipGetLastError();
}

// mfma: 0 = thin kernel, else the matrix-core precision (TN_MFMA_*) used
// when the op is eligible (the autotuner may choose thin for a shape class).
// tabs: the batch's table array (the op's tables at op.tab / op.tabB).
hipError_t level_op(int dtype, const LevelArgs &a, const DOp &op, const int32_t *tabs, int mfma, hipStream_t st) {
  if (mfma && mfma_eligible(dtype, op)) return mfma_contract(a, op, tabs + op.tab, mfma, st);
  return dtype == TN_C128 ? level_op_t<double2>(a, op, tabs, st) : level_op_t<float2>(a, op, tabs, st);
}

// One grouped launch of thin contractions and leaf adjoints: n items
// (device array; blk: their first-workgroup indices, ascending from 0) on
// `blocks` workgroups.
hipError_t level_group(int dtype, const LItem *items, const int32_t *blk, int n, int blocks, void *arena, int n_sets,
                       const int32_t *tabs, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (dtype == TN_C128)
    hipLaunchKernelGGL(level_group_contract_kernel<double2>, dim3(blocks), dim3(256), 0, st, items, blk, n,
                       (double2 *)arena, n_sets, tabs);
  else
    hipLaunchKernelGGL(level_group_contract_kernel<float2>, dim3(blocks), dim3(256), 0, st, items, blk, n,
                       (float2 *)arena, n_sets, tabs);
  return hipGetLastError();
}

hipError_t level_setup(int dtype, const LevelArgs &a, const void *consts, int n_const, const DParam *pt, int n_pt,
                       const void *bound, int per_set, int set0, int zero_begin, int zero_n, hipStream_t st) {
  int64_t per = n_const;
  dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (per + zero_n + 255) / 256 + 1)), a.n_sets);
  if (dtype == TN_C128)
    hipLaunchKernelGGL(level_setup_kernel<double2>, grid, dim3(256), 0, st, a, (const double2 *)consts, n_const, pt,
                       n_pt, (const double2 *)bound, per_set, set0, zero_begin, zero_n);
  else
    hipLaunchKernelGGL(level_setup_kernel<float2>, grid, dim3(256), 0, st, a, (const float2 *)consts, n_const, pt, n_pt,
                       (const float2 *)bound, per_set, set0, zero_begin, zero_n);
  return hipGetLastError();
}

hipError_t level_finish(int dtype, const LevelArgs &a, const DParam *pt, int n_pt, const void *dbound, int per_set,
                        int set0, int net, int n_sets_total, int n_params, double *out_val, double *out_grad,
                        int with_grad, hipStream_t st) {
  if (dtype == TN_C128)
    hipLaunchKernelGGL(level_finish_kernel<double2>, dim3(a.n_sets), dim3(256), 0, st, a, pt, n_pt,
                       (const double2 *)dbound, per_set, set0, net, n_sets_total, n_params, out_val, out_grad,
                       with_grad);
  else
    hipLaunchKernelGGL(level_finish_kernel<float2>, dim3(a.n_sets), dim3(256), 0, st, a, pt, n_pt,
                       (const float2 *)dbound, per_set, set0, net, n_sets_total, n_params, out_val, out_grad,
                       with_grad);
  return hipGetLastError();
}

}  // namespace qtn
