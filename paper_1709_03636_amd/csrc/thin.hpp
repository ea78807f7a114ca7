// Thin contractions and leaf adjoints on a level arena (device code shared by
// the grouped launches of level.hip and the per-step launches of mfma.hip):
// free-index deposit plus a per-op offset table for the summed index
// (eq. (1)), one or four outputs per lane, or several lanes per output.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
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
  if (nS == 0) return make_int2(0, 0);  // the one entry of an empty summed index (no load)
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

// One item of a grouped launch of thin contractions and leaf adjoints
// (rank / count: this workgroup's place among the item's workgroups): one
// op of one network, with the addressing of level_contract_kernel
// (level_leafgrad_kernel) inside the network's own arena region. A thin
// contraction's output is summed by L = 2^lgl adjacent lanes (summed entries
// k = part, part + L, ...; then a butterfly over the L lanes), so that steps
// with few outputs and long sums still fill the chip. All L lanes of an
// output are in the same loop iteration: the stride is a multiple of 256 and
// the total a multiple of L. Steps with many outputs give a lane four of
// them instead: lgl = -1 four consecutive ones (at least 2 Y-only bits),
// -2 / -3 four 64 apart along Y / X (thin_output4s).
template <typename V>
__device__ __forceinline__ void thin_item(const LItem &it, int rank, int count, V *arena, int n_sets,
                                          const int32_t *__restrict__ tabs) {
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

}  // namespace qtn
