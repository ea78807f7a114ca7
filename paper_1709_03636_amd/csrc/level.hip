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

namespace qtn {

template <typename T> struct LCplx;
template <> struct LCplx<float> { using type = float2; };
template <> struct LCplx<double> { using type = double2; };

__device__ __forceinline__ float2 l_fma(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 l_fma(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 l_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 l_d2(double2 v) { return v; }
template <typename V> __device__ __forceinline__ V l_from(double2 v);
template <> __device__ __forceinline__ float2 l_from<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 l_from<double2>(double2 v) { return v; }


__device__ __forceinline__ int2 l_tab(const int32_t *__restrict__ tb, int nS, int k) {
  if (nS <= kTabLoBits) return make_int2(tb[2 * k], tb[2 * k + 1]);
  const int lo = k & ((1 << kTabLoBits) - 1), hi = k >> kTabLoBits;
  const int32_t *h = tb + (2 << kTabLoBits);
  return make_int2(tb[2 * lo] + h[2 * hi], tb[2 * lo + 1] + h[2 * hi + 1]);
}

__device__ __forceinline__ uint32_t l_pdep(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    uint32_t low = mask & (0u - mask);
    if (v & 1u) r |= low;
    v >>= 1;
    mask ^= low;
  }
  return r;
}


__device__ __forceinline__ uint32_t l_deposit(uint32_t v, const int32_t runs[4], uint32_t mask) {
  if (runs[0] < 0) return l_pdep(v, mask);
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t shift = runs[j] & 0xff, len = (runs[j] >> 8) & 0xff, pos = (uint32_t)runs[j] >> 16;
    r |= __builtin_amdgcn_ubfe(v, shift, len) << pos;
  }
  return r;
}

// Partial sum of output c of a contraction on one parameter vector's slice:
// summed entries k = part, part + L, ...; the output index c = (i, b, j)
// holds the X-only bits, the batch bits (offset table) and the Y-only bits.
template <typename V>
__device__ __forceinline__ V thin_output(const V *base, const DOp &op, const DRuns &ru, const int32_t *__restrict__ tab,
                                         const int32_t *__restrict__ tabB, uint32_t c, int part, int L) {
  const uint32_t rest = c >> op.nFY;
  uint32_t bx = 0, by = 0;
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    bx = tabB[2 * b];
    by = tabB[2 * b + 1];
  }
  const V *X = base + op.x + l_deposit(rest >> op.nB, ru.runsX, op.maskX) + bx;
  const V *Y = base + op.y + l_deposit(c & ((1u << op.nFY) - 1u), ru.runsY, op.maskY) + by;
  V acc;
  acc.x = 0;
  acc.y = 0;
  const int K = 1 << op.nS;
  if (K >= 4 * L) {
    // four summed entries per iteration: their table and operand loads are
    // issued together (a lane's entries number a multiple of four)
    for (int k = part; k < K; k += 4 * L) {
      int2 t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] = l_tab(tab, op.nS, k + u * L);
      V x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = X[t[u].x];
        y[u] = Y[t[u].y];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = l_fma(acc, x[u], y[u]);
    }
    return acc;
  }
  for (int k = part; k < K; k += L) {
    const int2 t = l_tab(tab, op.nS, k);
    acc = l_fma(acc, X[t.x], Y[t.y]);
  }
  return acc;
}

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

__device__ __forceinline__ float l_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double l_xor(double v, int m) { return __shfl_xor(v, m, 64); }

// Four consecutive outputs c0 .. c0+3 of one parameter vector (c0 a multiple
// of 4, at least 2 Y-only bits): they share the X row, and their Y columns
// sit at fixed offsets deposit(r) from the first (disjoint bits add), so one
// X read serves four products.
template <typename V>
__device__ __forceinline__ void thin_output4(V *base, const DOp &op, const DRuns &ru, const int32_t *__restrict__ tab,
                                            const int32_t *__restrict__ tabB, uint32_t c0) {
  const uint32_t rest = c0 >> op.nFY;
  uint32_t bx = 0, by = 0;
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    bx = tabB[2 * b];
    by = tabB[2 * b + 1];
  }
  const V *X = base + op.x + l_deposit(rest >> op.nB, ru.runsX, op.maskX) + bx;
  const V *Y = base + op.y + l_deposit(c0 & ((1u << op.nFY) - 1u), ru.runsY, op.maskY) + by;
  uint32_t dy[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) dy[r] = l_deposit((uint32_t)r, ru.runsY, op.maskY);
  V acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    acc[r].x = 0;
    acc[r].y = 0;
  }
  const int K = 1 << op.nS;
  int k = 0;
  // two summed entries per iteration: ten operand loads in flight
  for (; k + 2 <= K; k += 2) {
    const int2 t0 = l_tab(tab, op.nS, k), t1 = l_tab(tab, op.nS, k + 1);
    const V x0 = X[t0.x], x1 = X[t1.x];
    V y0[4], y1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      y0[r] = Y[t0.y + dy[r]];
      y1[r] = Y[t1.y + dy[r]];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = l_fma(l_fma(acc[r], x0, y0[r]), x1, y1[r]);
  }
  if (k < K) {
    const int2 t = l_tab(tab, op.nS, k);
    const V x = X[t.x];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = l_fma(acc[r], x, Y[t.y + dy[r]]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) base[op.z + c0 + r] = acc[r];
}

// Four outputs c0 + 64 r (r < 4) of one parameter vector, c0 mod 256 < 64:
// bits 6-7 of the output index pick the four, and they are Y-only bits
// (ALONG_X false: at least 8 Y-only bits) or X-only bits (ALONG_X true: no
// Y-only or batch bits), so the four share the other operand's entry and
// their own entries sit at fixed offsets deposit(64 r). Consecutive lanes
// take consecutive c0: every load and store instruction is coalesced.
template <typename V, bool ALONG_X>
__device__ __forceinline__ void thin_output4s(V *base, const DOp &op, const DRuns &ru, const int32_t *__restrict__ tab,
                                             const int32_t *__restrict__ tabB, uint32_t c0) {
  uint32_t bx = 0, by = 0, fx, fy;
  if (ALONG_X) {
    fx = c0;
    fy = 0;
  } else {
    const uint32_t rest = c0 >> op.nFY;
    if (op.nB) {
      const uint32_t b = rest & ((1u << op.nB) - 1u);
      bx = tabB[2 * b];
      by = tabB[2 * b + 1];
    }
    fx = rest >> op.nB;
    fy = c0 & ((1u << op.nFY) - 1u);
  }
  const V *X = base + op.x + l_deposit(fx, ru.runsX, op.maskX) + bx;
  const V *Y = base + op.y + l_deposit(fy, ru.runsY, op.maskY) + by;
  uint32_t d[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    d[r] = ALONG_X ? l_deposit(64u * r, ru.runsX, op.maskX) : l_deposit(64u * r, ru.runsY, op.maskY);
  V acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    acc[r].x = 0;
    acc[r].y = 0;
  }
  for (int k = 0; k < (1 << op.nS); ++k) {
    const int2 t = l_tab(tab, op.nS, k);
    V v[4];
    if (ALONG_X) {
      const V y = Y[t.y];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = X[t.x + d[r]];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = l_fma(acc[r], v[r], y);
    } else {
      const V x = X[t.x];
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = Y[t.y + d[r]];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = l_fma(acc[r], x, v[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) base[op.z + c0 + 64u * r] = acc[r];
}

// Thin contractions and leaf adjoints of several networks at once: each item
// is one op of one network, with the addressing of level_contract_kernel
// (level_leafgrad_kernel) inside the network's own arena region. A thin
// contraction's output is summed by L = 2^lgl adjacent lanes (summed entries k = part, part + L, ...; then a butterfly over the
// L lanes), so that steps with few outputs and long sums still fill the
// chip. All L lanes of an output are in the same loop iteration: the
// stride is a multiple of 256 and the total a multiple of L. Steps with many
// outputs give a lane four of them instead: lgl = -1 four consecutive ones
// (at least 2 Y-only bits), -2 / -3 four 64 apart along Y / X
// (thin_output4s).
template <typename V>
__global__ __launch_bounds__(256) void level_group_contract_kernel(const LItem *__restrict__ items,
                                                                   const int32_t *__restrict__ blk, int n, V *arena,
                                                                   int n_sets, const int32_t *__restrict__ tabs) {
  int rank, count;
  const LItem &it = items[group_item(blk, n, &rank, &count)];
  const DOp op = it.op;
  const int lgOut = op.nFX + op.nB + op.nFY;
  const int32_t *tab = tabs + op.tab;
  const int32_t *tabB = tabs + op.tabB;
  V *reg = arena + it.base;
  if (op.type == OP_LEAFGRAD) {  // leaf adjoint (level_leafgrad_kernel per item)
    const int m = 1 << op.nFX;
    const int64_t tot = (int64_t)m * n_sets;
    for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < tot; g += (int64_t)count * 256) {
      const int64_t set = g >> op.nFX;
      const int i = (int)(g & (m - 1));
      V *base = reg + set * it.stride;
      V v = base[op.y + tab[i]];
      const V x = base[op.x + i];
      v.x += x.x;
      v.y += x.y;
      base[op.y + tab[i]] = v;
    }
    return;
  }
  if (it.lgl <= -2) {  // four outputs 64 apart per lane (lgOut >= 8)
    const int64_t nq = (int64_t)1 << (lgOut - 2);
    const int64_t total4 = nq * n_sets;
    for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < total4; g += (int64_t)count * 256) {
      const int64_t set = g >> (lgOut - 2);
      const uint32_t q = (uint32_t)(g & (nq - 1));
      const uint32_t c0 = ((q >> 6) << 8) | (q & 63u);
      if (it.lgl == -3)
        thin_output4s<V, true>(reg + set * it.stride, op, it.ru, tab, tabB, c0);
      else
        thin_output4s<V, false>(reg + set * it.stride, op, it.ru, tab, tabB, c0);
    }
    return;
  }
  if (it.lgl < 0) {  // four outputs per lane (nFY >= 2, so lgOut >= 2)
    const int64_t nq = (int64_t)1 << (lgOut - 2);
    const int64_t total4 = nq * n_sets;
    for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < total4; g += (int64_t)count * 256) {
      const int64_t set = g >> (lgOut - 2);
      const uint32_t c0 = (uint32_t)(g & (nq - 1)) << 2;
      thin_output4(reg + set * it.stride, op, it.ru, tab, tabB, c0);
    }
    return;
  }
  const int lgl = it.lgl;
  const int L = 1 << lgl;
  const int64_t nOut = (int64_t)1 << lgOut;
  const int64_t total = (nOut * n_sets) << lgl;
  for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < total; g += (int64_t)count * 256) {
    const int part = (int)(g & (L - 1));
    const int64_t o = g >> lgl;
    const int64_t set = o >> lgOut;
    const uint32_t c = (uint32_t)(o & (nOut - 1));
    V *base = reg + set * it.stride;
    V acc = thin_output(base, op, it.ru, tab, tabB, c, part, L);
    for (int m = 1; m < L; m <<= 1) {
      acc.x += l_xor(acc.x, m);
      acc.y += l_xor(acc.y, m);
    }
    if (part == 0) base[op.z + c] = acc;
  }
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
