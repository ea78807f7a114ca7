// Lane-record contractions shared by the fused executor and the level task
// executor: one 64-lane wave forms a small contraction (eq. (1)) whose
// per-lane operand offsets and summed-index offsets the host precomputed
// (the record layouts are described at kRecLanes), in a memory that holds
// every operand (LDS). Also the complex helpers and fixed-order cross-lane
// sums they use.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace qtn {

__device__ __forceinline__ float2 cmul_add(float2 acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ double2 cmul_add(double2 acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
template <typename V> __device__ __forceinline__ V czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Cross-lane moves with DPP (no LDS traffic). Inside a row of 16 lanes the
// controls used are permutations of the row; row_bcast15 / row_bcast31 add
// the last lane of a row into the rows selected by the row mask (the other
// rows receive 0).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float2 dpp_c(float2 v) {
  return make_float2(dpp_f32<CTRL, ROWS>(v.x), dpp_f32<CTRL, ROWS>(v.y));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double2 dpp_c(double2 v) {
  return make_double2(dpp_f64<CTRL, ROWS>(v.x), dpp_f64<CTRL, ROWS>(v.y));
}

// Sum over aligned groups of 2^lg lanes (lg <= 6), fixed order: lanes 1
// apart, 2 apart (quad permutations), the mirrored half-row and row, then
// rows pairwise and the two row pairs. For lg <= 4 every lane of a group
// holds the group's sum afterwards; in any case its last lane does. All 64
// lanes must be active.
template <typename V>
__device__ __forceinline__ V group_sum(V v, int lg) {
  if (lg > 0) v = cadd(v, dpp_c<0xB1>(v));        // quad_perm [1,0,3,2]
  if (lg > 1) v = cadd(v, dpp_c<0x4E>(v));        // quad_perm [2,3,0,1]
  if (lg > 2) v = cadd(v, dpp_c<0x141>(v));       // row_half_mirror
  if (lg > 3) v = cadd(v, dpp_c<0x140>(v));       // row_mirror
  if (lg > 4) v = cadd(v, dpp_c<0x142, 0xA>(v));  // row_bcast15 into rows 1, 3
  if (lg > 5) v = cadd(v, dpp_c<0x143, 0xC>(v));  // row_bcast31 into rows 2, 3
  return v;
}

__device__ __forceinline__ double group_sum_f64(double v, int lg) {
  if (lg > 0) v += dpp_f64<0xB1>(v);
  if (lg > 1) v += dpp_f64<0x4E>(v);
  if (lg > 2) v += dpp_f64<0x141>(v);
  if (lg > 3) v += dpp_f64<0x140>(v);
  if (lg > 4) v += dpp_f64<0x142, 0xA>(v);
  if (lg > 5) v += dpp_f64<0x143, 0xC>(v);
  return v;
}

// Small contraction from a lane record (64-lane workgroups): the lane's
// operand offsets and the summed-index table come precomputed, the table is
// read out of the record lanes into scalar registers.
template <typename V, int LGK>
__device__ __forceinline__ void contract_lite(const V *xm, const V *ym, V *zm, const int4 &rec, uint32_t hdr) {
  constexpr int K = 1 << LGK;
  const int nOut = 1 << ((hdr >> 7) & 15u);
  const int z = (int)(hdr >> 15);
  int32_t tx[K], ty[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_readlane(rec.z, k);
    tx[k] = (int32_t)(t & 0xffffu);
    ty[k] = (int32_t)(t >> 16);
  }
  if ((int)(threadIdx.x & 63) < nOut) {
    V xv[K], yv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      xv[k] = xm[rec.x + tx[k]];
      yv[k] = ym[rec.y + ty[k]];
    }
    V acc = czero<V>();
#pragma unroll
    for (int k = 0; k < K; ++k) acc = cmul_add(acc, xv[k], yv[k]);
    zm[z + (threadIdx.x & 63)] = acc;
  }
}
template <typename V, int LGK>
__device__ __forceinline__ void contract_lite(V *mem, const int4 &rec, uint32_t hdr) {
  contract_lite<V, LGK>(mem, mem, mem, rec, hdr);
}

// Outer product (no summed index) with up to 256 outputs from a lane
// record: lane l forms outputs l + 64 r, whose operand offsets differ from
// output l's by the uniform steps held in the record.
template <typename V>
__device__ __forceinline__ void contract_wide(const V *xm, const V *ym, V *zm, const int4 &rec, uint32_t hdr) {
  const int R = 1 << (((hdr >> 7) & 15u) - 6);
  const int z = (int)(hdr >> 15) + (int)(threadIdx.x & 63);
  int32_t dx[4], dy[4];
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const uint32_t t = (uint32_t)__builtin_amdgcn_readlane(rec.w, r);
    dx[r] = (int32_t)(t & 0xffffu);
    dy[r] = (int32_t)(t >> 16);
  }
  V xv[4], yv[4];
  xv[0] = xm[rec.x];
  yv[0] = ym[rec.y];
#pragma unroll
  for (int r = 1; r < 4; ++r)
    if (r < R) {
      xv[r] = xm[rec.x + dx[r]];
      yv[r] = ym[rec.y + dy[r]];
    }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (r < R) zm[z + 64 * r] = cmul_add(czero<V>(), xv[r], yv[r]);
}
template <typename V>
__device__ __forceinline__ void contract_wide(V *mem, const int4 &rec, uint32_t hdr) {
  contract_wide<V>(mem, mem, mem, rec, hdr);
}


// Contraction with few outputs and many summed entries from a lane record:
// G lanes per output each sum R entries (uniform offset steps), then the G
// partial sums are reduced across lanes in a fixed order.
template <typename V>
__device__ __forceinline__ void contract_narrow(const V *xm, const V *ym, V *zm, const int4 &rec, uint32_t hdr) {
  const int lgG = (int)((hdr >> 3) & 15u);
  const int nOut = 1 << ((hdr >> 7) & 15u);
  const int R = 1 << ((hdr >> 11) & 15u);
  const int z = (int)(hdr >> 15);
  V acc = czero<V>();
  for (int i = 0; i < R; i += 4) {
    V xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < R) {
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane(rec.z, i + u);
        xv[u] = xm[rec.x + (int32_t)(t & 0xffffu)];
        yv[u] = ym[rec.y + (int32_t)(t >> 16)];
      }
  #pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < R) acc = cmul_add(acc, xv[u], yv[u]);
  }
  acc = group_sum(acc, lgG);  // valid in the last lane of each group
  const int l = (int)(threadIdx.x & 63), g1 = (1 << lgG) - 1;
  if ((l & g1) == g1 && (l >> lgG) < nOut) zm[z + (l >> lgG)] = acc;
}
template <typename V>
__device__ __forceinline__ void contract_narrow(V *mem, const int4 &rec, uint32_t hdr) {
  contract_narrow<V>(mem, mem, mem, rec, hdr);
}

// kRecAcc (task executor): a leaf adjoint of 2^B <= 256 entries added into
// its parametric tensor's accumulator in canonical layout: lane l adds
// entries l + 64 q (offset x of entry l, canonical indices packed 8 bits
// each in y) to the accumulator at the header's offset. The canonical map
// is a permutation, so no two lanes write the same entry.
template <typename V>
__device__ __forceinline__ void acc_rec(const V *xm, V *zm, const int4 &rec, uint32_t hdr) {
  const int cnt = 1 << ((hdr >> 7) & 15u);
  const int z = (int)(hdr >> 15);
  const int l = (int)(threadIdx.x & 63);
  V xv[4], zv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (l + 64 * q < cnt) {
      xv[q] = xm[rec.x + 64 * q];
      zv[q] = zm[z + (((uint32_t)rec.y >> (8 * q)) & 0xffu)];
    }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (l + 64 * q < cnt) zm[z + (((uint32_t)rec.y >> (8 * q)) & 0xffu)] = cadd(zv[q], xv[q]);
}

}  // namespace qtn
