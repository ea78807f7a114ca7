// Device code of the level executor's items (device.hpp, PItem): one
// workgroup of 256 threads runs task `rank` of `count` of an item. The same
// bodies serve the item kernels (one item per launch, rank = workgroup) and
// the task executor (one workgroup runs every rank of a one-vector item).
//
// Every buffer of a (network, parameter vector) pair lives in the network's
// region of a global-memory arena, with the fused executor's addressing:
// free-index bits deposited into the operands, a per-op offset table for the
// summed index (eq. (1)).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "kargs.hpp"
#include "tile.hpp"

namespace qtn {

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

// Offsets of summed entry k from packed bit positions (5 bits each, lowest
// summed bit first; at most kPackedTabBits bits).
__device__ __forceinline__ int2 l_ptab(uint32_t px, uint32_t py, int nS, int k) {
  int ox = 0, oy = 0;
#pragma unroll
  for (int t = 0; t < kPackedTabBits; ++t)
    if (t < nS) {
      const int b = (k >> t) & 1;
      ox |= b << ((px >> (5 * t)) & 31);
      oy |= b << ((py >> (5 * t)) & 31);
    }
  return make_int2(ox, oy);
}

// Summed-index offsets of an op: packed positions (pk.x, pk.y) when pk.z,
// else its table.
__device__ __forceinline__ int2 l_koff(const int32_t *__restrict__ tb, const int3 &pk, int nS, int k) {
  return pk.z ? l_ptab((uint32_t)pk.x, (uint32_t)pk.y, nS, k) : l_tab(tb, nS, k);
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

__device__ __forceinline__ float l_xor(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double l_xor(double v, int m) { return __shfl_xor(v, m, 64); }

// Partial sum of output c of a contraction on one parameter vector's slice:
// summed entries k = part, part + L, ...; the output index c = (i, b, j)
// holds the X-only bits, the batch bits (offset table) and the Y-only bits.
template <typename V>
__device__ __forceinline__ V thin_output(const V *xb, const V *yb, const DOp &op, const DRuns &ru,
                                         const int32_t *__restrict__ tab, const int3 &pk,
                                         const int32_t *__restrict__ tabB, uint32_t c, int part, int L) {
  const uint32_t rest = c >> op.nFY;
  uint32_t bx = 0, by = 0;
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    bx = tabB[2 * b];
    by = tabB[2 * b + 1];
  }
  const V *X = xb + op.x + l_deposit(rest >> op.nB, ru.runsX, op.maskX) + bx;
  const V *Y = yb + op.y + l_deposit(c & ((1u << op.nFY) - 1u), ru.runsY, op.maskY) + by;
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
      for (int u = 0; u < 4; ++u) t[u] = l_koff(tab, pk, op.nS, k + u * L);
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
    const int2 t = l_koff(tab, pk, op.nS, k);
    acc = l_fma(acc, X[t.x], Y[t.y]);
  }
  return acc;
}

// Four consecutive outputs c0 .. c0+3 of one parameter vector (c0 a multiple
// of 4, at least 2 Y-only bits): they share the X row, and their Y columns
// sit at fixed offsets deposit(r) from the first (disjoint bits add), so one
// X read serves four products.
template <typename V>
__device__ __forceinline__ void thin_output4(const V *xb, const V *yb, V *zb, const DOp &op, const DRuns &ru,
                                            const int32_t *__restrict__ tab, const int3 &pk,
                                            const int32_t *__restrict__ tabB, uint32_t c0) {
  const uint32_t rest = c0 >> op.nFY;
  uint32_t bx = 0, by = 0;
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    bx = tabB[2 * b];
    by = tabB[2 * b + 1];
  }
  const V *X = xb + op.x + l_deposit(rest >> op.nB, ru.runsX, op.maskX) + bx;
  const V *Y = yb + op.y + l_deposit(c0 & ((1u << op.nFY) - 1u), ru.runsY, op.maskY) + by;
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
    const int2 t0 = l_koff(tab, pk, op.nS, k), t1 = l_koff(tab, pk, op.nS, k + 1);
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
    const int2 t = l_koff(tab, pk, op.nS, k);
    const V x = X[t.x];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = l_fma(acc[r], x, Y[t.y + dy[r]]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) zb[op.z + c0 + r] = acc[r];
}

// Four outputs c0 + 64 r (r < 4) of one parameter vector, c0 mod 256 < 64:
// bits 6-7 of the output index pick the four, and they are Y-only bits
// (ALONG_X false: at least 8 Y-only bits) or X-only bits (ALONG_X true: no
// Y-only or batch bits), so the four share the other operand's entry and
// their own entries sit at fixed offsets deposit(64 r). Consecutive lanes
// take consecutive c0: every load and store instruction is coalesced.
template <typename V, bool ALONG_X>
__device__ __forceinline__ void thin_output4s(const V *xb, const V *yb, V *zb, const DOp &op, const DRuns &ru,
                                             const int32_t *__restrict__ tab, const int3 &pk,
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
  const V *X = xb + op.x + l_deposit(fx, ru.runsX, op.maskX) + bx;
  const V *Y = yb + op.y + l_deposit(fy, ru.runsY, op.maskY) + by;
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
    const int2 t = l_koff(tab, pk, op.nS, k);
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
  for (int r = 0; r < 4; ++r) zb[op.z + c0 + 64u * r] = acc[r];
}

// PK_THIN: a thin contraction or a leaf adjoint over the pass's parameter
// vectors. A thin contraction's output is summed by L = 2^lgl adjacent lanes
// (summed entries k = part, part + L, ...; then a butterfly over the L
// lanes), so that steps with few outputs and long sums still fill the chip.
// All L lanes of an output are in the same loop iteration: the stride is a
// multiple of 256 and the total a multiple of L. Steps with many outputs give
// a lane four of them instead: lgl = -1 four consecutive ones (at least 2
// Y-only bits), -2 / -3 four 64 apart along Y / X (thin_output4s). A leaf
// adjoint adds the adjoint of a parametric leaf into the tensor's
// canonical-layout accumulator at y (the table maps buffer to canonical index).
// LDSOK (task executor): operands flagged in it.a0 (kLdsX / kLdsY / kLdsZ)
// are read from / written to the workgroup's LDS arena `lar` instead of the
// region, and kPackedTab items take their summed-index offsets from packed
// bit positions instead of the table.
// FL: the item's operands in LDS (kLdsX / kLdsY / kLdsZ, the item's a0 &
// 7) as a compile-time set, so every access is an LDS or a global access
// rather than a generic one.
template <typename V, bool LDSOK, int FL>
__device__ __forceinline__ void task_thin(const PItem &it, int rank, int count, V *arena, V *lar, int n_sets,
                                          const int32_t *__restrict__ tabs) {
  const DOp &op = it.op;
  const int lgOut = op.nFX + op.nB + op.nFY;
  const int32_t *tab = tabs + op.tab;
  const int32_t *tabB = tabs + op.tabB;
  const int fl = LDSOK ? it.a0 : 0;
  const int3 pk = make_int3(it.a1, it.a2, fl & kPackedTab);
  V *reg = arena + it.base;
  auto pick = [&](V *base, int bit) { return LDSOK && (FL & bit) ? lar : base; };
  if (op.type == OP_LEAFGRAD) {
    const int m = 1 << op.nFX;
    const int64_t tot = (int64_t)m * n_sets;
    for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < tot; g += (int64_t)count * 256) {
      const int64_t set = g >> op.nFX;
      const int i = (int)(g & (m - 1));
      V *base = reg + set * it.stride;
      V *acc = pick(base, kLdsY);
      V v = acc[op.y + tab[i]];
      const V x = pick(base, kLdsX)[op.x + i];
      v.x += x.x;
      v.y += x.y;
      acc[op.y + tab[i]] = v;
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
      V *base = reg + set * it.stride;
      if (it.lgl == -3)
        thin_output4s<V, true>(pick(base, kLdsX), pick(base, kLdsY), pick(base, kLdsZ), op, it.ru, tab, pk, tabB, c0);
      else
        thin_output4s<V, false>(pick(base, kLdsX), pick(base, kLdsY), pick(base, kLdsZ), op, it.ru, tab, pk, tabB, c0);
    }
    return;
  }
  if (it.lgl < 0) {  // four consecutive outputs per lane (nFY >= 2, so lgOut >= 2)
    const int64_t nq = (int64_t)1 << (lgOut - 2);
    const int64_t total4 = nq * n_sets;
    for (int64_t g = rank * (int64_t)256 + threadIdx.x; g < total4; g += (int64_t)count * 256) {
      const int64_t set = g >> (lgOut - 2);
      const uint32_t c0 = (uint32_t)(g & (nq - 1)) << 2;
      V *base = reg + set * it.stride;
      thin_output4(pick(base, kLdsX), pick(base, kLdsY), pick(base, kLdsZ), op, it.ru, tab, pk, tabB, c0);
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
    V acc = thin_output(pick(base, kLdsX), pick(base, kLdsY), op, it.ru, tab, pk, tabB, c, part, L);
    for (int m = 1; m < L; m <<= 1) {
      acc.x += l_xor(acc.x, m);
      acc.y += l_xor(acc.y, m);
    }
    if (part == 0) pick(base, kLdsZ)[op.z + c] = acc;
  }
}

// PK_MFMA: one output tile of one summed-index range of one parameter
// vector: rank = (set, range, tile) with the tile fastest. An item with
// lgl > 0 (split summed index) writes partial tiles to the split scratch
// ([set][range][M x N] from element zs), else the result tile in place.
template <int PREC, bool XK, bool YK, int BM, int BN, bool DB>
__device__ __forceinline__ void task_mfma_t(char *lds, const PItem &it, int rank, const LvlArgs &a) {
  using T = TileT<BM, BN>;
  constexpr int eb = elem_bytes(PREC);
  const DOp &op = it.op;
  const int lt = (op.nFX > T::LM ? op.nFX - T::LM : 0) + (op.nFY > T::LN ? op.nFY - T::LN : 0);  // log2 tiles per set
  const int ls = it.lgl;
  const int set = rank >> (lt + ls), part = (rank >> lt) & ((1 << ls) - 1), tile = rank & ((1 << lt) - 1);
  if (set >= a.n_sets) return;
  char *base = (char *)a.arena + (it.base + (int64_t)set * it.stride) * eb;
  const int kl = op.nS - ls;
  char *z = ls == 0 ? base + (int64_t)op.z * eb
                    : (char *)a.split + (it.zs + ((((int64_t)set << ls) + part) << (op.nFX + op.nFY))) * eb;
  // one-item launches (the item kernel) have LDS for two tile buffers
  const int32_t *pk = (it.mv & kMfmaPacked) ? &it.a0 : nullptr;  // a0 .. a5: packed summed-bit positions
  any_tile<PREC, XK, YK, BM, BN, DB>(lds, base, op, it.ru, a.tabs + op.tab, pk, tile, part << kl, (part + 1) << kl, z);
}

// Kernel variant of a matrix-core item: bit 0 XK (X's lowest address bit is
// summed), bit 1 YK, bit 2 BM = 16, bit 3 BN = 16 (the precision is the
// kernel's).
template <int PREC, bool DB>
__device__ __forceinline__ void task_mfma(char *lds, const PItem &it, int rank, const LvlArgs &a) {
#define QTN_TV(XK, YK, BM, BN) \
  case (XK ? 1 : 0) | (YK ? 2 : 0) | (BM == 16 ? 4 : 0) | (BN == 16 ? 8 : 0): \
    task_mfma_t<PREC, XK, YK, BM, BN, DB>(lds, it, rank, a);                   \
    return;
#define QTN_TV4(BM, BN) QTN_TV(false, false, BM, BN) QTN_TV(true, false, BM, BN) QTN_TV(false, true, BM, BN) \
  QTN_TV(true, true, BM, BN)
  if constexpr (PREC == TN_MFMA_FP64) {
    switch (it.mv & 15) { QTN_TV4(64, 64) default: return; }
  } else {
    switch (it.mv & 15) {
      QTN_TV4(64, 64)
      QTN_TV4(16, 64)
      QTN_TV4(64, 16)
      default:
        return;
    }
  }
#undef QTN_TV4
#undef QTN_TV
}

// PK_SPLITSUM: Z[i] = sum over ranges r in order of split[zs + ((set 2^lgl
// + r) M N) + i], in FP64.
template <typename V>
__device__ __forceinline__ void task_splitsum(const PItem &it, int rank, int count, const LvlArgs &a) {
  const int ls = it.lgl, lmn = it.op.nFX + it.op.nFY;
  const int64_t total = (int64_t)a.n_sets << lmn;
  const V *sp = reinterpret_cast<const V *>(a.split) + it.zs;
  V *ar = reinterpret_cast<V *>(a.arena);
  for (int64_t g = (int64_t)rank * 256 + threadIdx.x; g < total; g += (int64_t)count * 256) {
    const int64_t set = g >> lmn, i = g & ((int64_t(1) << lmn) - 1);
    const V *src = sp + ((set << ls) << lmn) + i;
    double re = 0.0, im = 0.0;
    for (int r = 0; r < (1 << ls); ++r) {
      const V v = src[(int64_t)r << lmn];
      re += v.x;
      im += v.y;
    }
    ar[it.base + set * it.stride + it.op.z + i] = l_from<V>(make_double2(re, im));
  }
}

// Sum over the 256 threads of a workgroup in FP64 (fixed tree; `red` holds
// 8 doubles of LDS); the result is valid in thread 0.
__device__ __forceinline__ double2 wg_sum2(double re, double im, double *red) {
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  __syncthreads();  // red may still be read by an earlier sum
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = re;
    red[4 + (threadIdx.x >> 6)] = im;
  }
  __syncthreads();
  return make_double2(red[0] + red[1] + red[2] + red[3], red[4] + red[5] + red[6] + red[7]);
}

// PK_SCALAR: rank-0 result in FP64. Task (set, g) of G = lgl workgroups per
// parameter vector sums the summed entries g*256 + t, g*256 + t + G*256, ...;
// with G = 1 the sum is the scalar, else it goes to the partial sums
// part[zs + set*G + g] and a PK_SCALAR_SUM item adds them in index order.
template <typename V>
__device__ __forceinline__ void task_scalar(char *lds, const PItem &it, int rank, const LvlArgs &a) {
  const int G = it.lgl;
  const int set = rank / G, g = rank - set * G;
  if (set >= a.n_sets) return;
  const DOp &op = it.op;
  const int32_t *tab = a.tabs + op.tab;
  const V *base = reinterpret_cast<const V *>(a.arena) + it.base + set * it.stride;
  const int64_t K = (int64_t)1 << op.nS;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int64_t k = g * 256 + threadIdx.x; k < K; k += (int64_t)G * 256) {
    const int2 o = l_tab(tab, op.nS, (int)k);
    const double2 x = l_d2(base[op.x + o.x]);
    const double2 y = l_d2(base[op.y + o.y]);
    re += x.x * y.x - x.y * y.y;
    im += x.x * y.y + x.y * y.x;
  }
  const double2 s = wg_sum2(re, im, reinterpret_cast<double *>(lds));
  if (threadIdx.x == 0) {
    double *dst = G == 1 ? a.scal + it.sbase + ((int64_t)set * it.n_comp + op.z) * 2 : a.part + it.zs + ((int64_t)set * G + g) * 2;
    dst[0] = s.x;
    dst[1] = s.y;
  }
}

// PK_SCALAR_SUM: the G = a0 partial sums of each parameter vector, in order.
__device__ __forceinline__ void task_scalar_sum(const PItem &it, int rank, const LvlArgs &a) {
  const int set = rank * 256 + (int)threadIdx.x;
  if (set >= a.n_sets) return;
  const int G = it.a0;
  double re = 0.0, im = 0.0;
  for (int g = 0; g < G; ++g) {
    re += a.part[it.zs + ((int64_t)set * G + g) * 2];
    im += a.part[it.zs + ((int64_t)set * G + g) * 2 + 1];
  }
  double *dst = a.scal + it.sbase + ((int64_t)set * it.n_comp + it.op.z) * 2;
  dst[0] = re;
  dst[1] = im;
}

// PK_SEED: adjoint seed of component op.aux0, the product of the other
// component scalars.
template <typename V>
__device__ __forceinline__ void task_seed(const PItem &it, int rank, const LvlArgs &a) {
  const int set = rank * 256 + (int)threadIdx.x;
  if (set >= a.n_sets) return;
  const double *sc = a.scal + it.sbase + (int64_t)set * it.n_comp * 2;
  double pr = 1.0, pi = 0.0;
  for (int j = 0; j < it.n_comp; ++j) {
    if (j == it.op.aux0) continue;
    const double nr = pr * sc[2 * j] - pi * sc[2 * j + 1], ni = pr * sc[2 * j + 1] + pi * sc[2 * j];
    pr = nr;
    pi = ni;
  }
  V *base = reinterpret_cast<V *>(a.arena) + it.base + set * it.stride;
  base[it.op.z] = l_from<V>(make_double2(pr, pi));
}

// PK_SETUP: task (set, chunk) of G = lgl chunks per parameter vector copies
// the constants (a1 entries from a0) and the bound parametric tensors
// (DParams a2 .. a2 + a3) into the vector's slice and clears the a5 adjoint
// accumulator entries from zs.
template <typename V>
__device__ __forceinline__ void task_setup(const PItem &it, int rank, const LvlArgs &a, V *lar) {
  const int G = it.lgl;
  const int set = rank / G, chunk = rank - set * G;
  if (set >= a.n_sets) return;
  V *base = reinterpret_cast<V *>(a.arena) + it.base + set * it.stride;
  const V *consts = reinterpret_cast<const V *>(a.consts) + it.a0;
  const int step = G * 256, first = chunk * 256 + (int)threadIdx.x;
  const bool mirror = lar && (it.mv & 1);  // task executor: the leaf region also into LDS
  for (int e = first; e < it.a1; e += step) {
    const V v = consts[e];
    base[e] = v;
    if (mirror) lar[e] = v;
  }
  const V *bs = reinterpret_cast<const V *>(a.bound) + (size_t)(a.set0 + set) * a.per_set;
  for (int t = 0; t < it.a3; ++t) {
    const DParam d = a.ptens[it.a2 + t];
    for (int e = first; e < (1 << d.bits); e += step) {
      const V v = bs[d.slot + e];
      base[d.off + e] = v;
      if (mirror) lar[d.off + e] = v;
    }
  }
  V *zdst = lar && (it.mv & 2) ? lar + it.a4 : base + it.zs;  // adjoint accumulators in LDS or the region
  for (int e = first; e < it.a5; e += step) {
    V z;
    z.x = 0;
    z.y = 0;
    zdst[e] = z;
  }
}

// PK_FINISH: task `set` writes the network's value (the product of its
// component scalars) and, with gradients, sum over its parametric tensors of
// coeff * Re <Gbar, dG/dtheta> per parameter, in FP64.
template <typename V>
__device__ __forceinline__ void task_finish(char *lds, const PItem &it, int rank, const LvlArgs &a, const V *lar) {
  const int set = rank;
  if (set >= a.n_sets) return;
  double *red = reinterpret_cast<double *>(lds);
  double *gacc = red + 8;
  const V *base = reinterpret_cast<const V *>(a.arena) + it.base + set * it.stride;
  const bool gl = lar && it.mv;  // adjoint accumulators (offsets goff) in LDS from a3
  const V *gb = gl ? lar : base;
  const int64_t g0 = gl ? it.a3 - it.zs : 0;
  const int gs = a.set0 + set, net = it.a0;
  if (threadIdx.x == 0) {
    const double *sc = a.scal + it.sbase + (int64_t)set * it.n_comp * 2;
    double pr = 1.0, pi = 0.0;
    for (int j = 0; j < it.n_comp; ++j) {
      const double nr = pr * sc[2 * j] - pi * sc[2 * j + 1], ni = pr * sc[2 * j + 1] + pi * sc[2 * j];
      pr = nr;
      pi = ni;
    }
    a.out_val[((size_t)net * a.n_sets_total + gs) * 2] = pr;
    a.out_val[((size_t)net * a.n_sets_total + gs) * 2 + 1] = pi;
  }
  if (!a.with_grad) return;
  const V *dset = reinterpret_cast<const V *>(a.dbound) + (size_t)gs * a.per_set;
  for (int p0 = 0; p0 < a.n_params; p0 += 64) {
    __syncthreads();
    for (int p = threadIdx.x; p < 64; p += blockDim.x) gacc[p] = 0.0;
    for (int t = 0; t < it.a2; ++t) {
      const DParam d = a.ptens[it.a1 + t];
      if (d.param < p0 || d.param >= p0 + 64) continue;
      double acc = 0.0;
      for (int e = threadIdx.x; e < (1 << d.bits); e += 256) {
        const double2 g = l_d2(gb[g0 + d.goff + e]);
        const double2 dv = l_d2(dset[d.slot + e]);
        acc += g.x * dv.x - g.y * dv.y;
      }
      const double2 s = wg_sum2(acc, 0.0, red);
      if (threadIdx.x == 0) gacc[d.param - p0] += d.coeff * s.x;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < 64 && p0 + p < a.n_params; p += blockDim.x)
      a.out_grad[((size_t)net * a.n_sets_total + gs) * a.n_params + p0 + p] = gacc[p];
  }
}

// Task `rank` of `count` of an item; PREC: the matrix-core precision
// (TN_MFMA_FP32 or TN_MFMA_BF16X3 for complex64, TN_MFMA_FP64 for
// complex128). lds: at least max(kTileLds<PREC>, 72 doubles), 16-byte aligned;
// twice kTileLds for split-BF16 items unless LDSOK (item kernel: double
// buffered tiles).
// lar: the task executor's LDS arena for small tensors (LDSOK), else unused.
template <int PREC, bool LDSOK>
__device__ __forceinline__ void run_item(char *lds, char *lar, const PItem &it, int rank, int count, const LvlArgs &a) {
  using V = typename std::conditional<PREC == TN_MFMA_FP64, double2, float2>::type;
  V *larv = LDSOK ? reinterpret_cast<V *>(lar) : nullptr;
  switch (it.kind) {
    case PK_SETUP: task_setup<V>(it, rank, a, larv); break;
    case PK_THIN: {
      V *ar = reinterpret_cast<V *>(a.arena);
      switch (LDSOK ? it.a0 & 7 : 0) {
        case 0: task_thin<V, LDSOK, 0>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 1: task_thin<V, LDSOK, 1>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 2: task_thin<V, LDSOK, 2>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 3: task_thin<V, LDSOK, 3>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 4: task_thin<V, LDSOK, 4>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 5: task_thin<V, LDSOK, 5>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        case 6: task_thin<V, LDSOK, 6>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
        default: task_thin<V, LDSOK, 7>(it, rank, count, ar, larv, a.n_sets, a.tabs); break;
      }
      break;
    }
    case PK_MFMA: task_mfma<PREC, !LDSOK>(lds, it, rank, a); break;
    case PK_SPLITSUM: task_splitsum<V>(it, rank, count, a); break;
    case PK_SCALAR: task_scalar<V>(lds, it, rank, a); break;
    case PK_SCALAR_SUM: task_scalar_sum(it, rank, a); break;
    case PK_SEED: task_seed<V>(it, rank, a); break;
    default: task_finish<V>(lds, it, rank, a, larv); break;
  }
}

}  // namespace qtn
