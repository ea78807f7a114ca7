// Complex GEMM tiles on the matrix cores (device code of the level
// executor's matrix-core items): eq. (1) as
//   Z[m*N + n] = sum_k X[rX(m) + tX(k)] * Y[tY(k) + cY(n)],
// with rX / cY the deposit of the free-index bits into X / Y and (tX, tY)
// the op's summed-index offsets. The bit permutation is applied while the
// tiles are staged into LDS, so X and Y are read in their stored layout.
//
// Complex products use four real products (4M) on v_mfma_f32_16x16x4_f32
// with FP32 accumulation for complex64 (or split-BF16 products, below), on
// v_mfma_f64_16x16x4_f64 with FP64 accumulation for complex128: with the
// summed index interleaved as (re, im) pairs, Re Z = [Xr, -Xi] . [Yr; Yi] and
// Im Z = [Xi, Xr] . [Yr; Yi]. Workgroup tile: BM x BN complex outputs
// (64 x 64, or 16 x 64 / 64 x 16 when one free index has only 2-5 bits) for
// four waves; 16 complex summed entries per LDS stage, the next stage
// prefetched into registers while the matrix cores work on the current one.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace qtn {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 real matrix product, FP32 or FP64: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; result entry r < 4 of lane l is D[row(l, r)][l % 16]
// with row = 4 (l / 16) + r for FP32 and row = l / 16 + 4 r for FP64
// (measured on gfx950).
__device__ __forceinline__ mf4 mfma4(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ md4 mfma4(double a, double b, md4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <typename V> struct Acc4;
template <> struct Acc4<float2> {
  using R = float;
  using type = mf4;
  static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};
template <> struct Acc4<double2> {
  using R = double;
  using type = md4;
  static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
};
__device__ __forceinline__ float2 make_c(float r, float i) { return make_float2(r, i); }
__device__ __forceinline__ double2 make_c(double r, double i) { return make_double2(r, i); }

namespace {

constexpr int BK = 16;

// Wave layout of a BM x BN tile: GM x GN waves, each WM x WN MFMA tiles of
// 16 x 16; NX / NY staged X / Y entries per thread and stage.
template <int BM, int BN>
struct TileT {
  static constexpr int LM = BM == 64 ? 6 : 4, LN = BN == 64 ? 6 : 4;
  static constexpr int GM = (BM == 64 && BN == 64) ? 2 : BM / 16;
  static constexpr int GN = 4 / GM;
  static constexpr int WM = BM / 16 / GM, WN = BN / 16 / GN;
  static constexpr int NX = BM / 16, NY = BN / 16;
  static constexpr int AS = BK + 1;  // LDS row stride of the X tile (complex), padded against bank conflicts
  static constexpr int BS = BN + 2;  // LDS row stride of the Y tile
  static constexpr int PS = BK + 4;  // packed-tile row stride (dwords), 16-byte aligned rows
  static_assert(GM * GN == 4 && WM >= 1 && WN >= 1, "tile");
};

__device__ __forceinline__ uint32_t g_pdep(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    uint32_t low = mask & (0u - mask);
    if (v & 1u) r |= low;
    v >>= 1;
    mask ^= low;
  }
  return r;
}

// Deposit of v's low bits at the set bits of mask, from the mask's runs of
// consecutive bits (DRuns encoding; runs[0] < 0: more than four runs, bit loop).
__device__ __forceinline__ uint32_t g_deposit(uint32_t v, const int32_t runs[4], uint32_t mask) {
  if (runs[0] < 0) return g_pdep(v, mask);
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t shift = runs[j] & 0xff, len = (runs[j] >> 8) & 0xff, pos = (uint32_t)runs[j] >> 16;
    r |= __builtin_amdgcn_ubfe(v, shift, len) << pos;
  }
  return r;
}

__device__ __forceinline__ int2 g_tab(const int32_t *__restrict__ tb, int nS, int k) {
  if (nS <= kTabLoBits) return make_int2(tb[2 * k], tb[2 * k + 1]);
  const int lo = k & ((1 << kTabLoBits) - 1), hi = k >> kTabLoBits;
  const int32_t *h = tb + (2 << kTabLoBits);
  return make_int2(tb[2 * lo] + h[2 * hi], tb[2 * lo + 1] + h[2 * hi + 1]);
}

// Staging assignment: each thread moves NX X and NY Y entries per stage.
// Summed-index offsets add over disjoint bits, so the offset of k0 + k (k0
// a multiple of BK, k < BK) is t(k0) + t(k): the per-thread parts t(k) are
// fixed, and t(k0) is one workgroup-uniform lookup per stage.
// XK: X's lowest address bit is summed (stage X with k fastest), else m
// fastest; YK likewise for Y. BLK (split-BF16 tiles, whose LDS rows are
// [row][k] with a 20-dword stride): with m (n) fastest, a wave stages a
// 16 x 4 block (16 consecutive rows, 128 contiguous bytes each, at 4 summed
// entries) instead of 64 rows at one summed entry, so its LDS writes fall
// on 64 different banks instead of 16.
template <bool XK, bool YK, int BM, int BN, typename V = float2, bool BLK = false>
struct Stager {
  using T = TileT<BM, BN>;
  int xr[T::NX], xk[T::NX], yk[T::NY], yn[T::NY];
  uint32_t xrow[T::NX], ycol[T::NY];
  V xv[T::NX], yv[T::NY];
  __device__ __forceinline__ Stager(const DOp &op, const DRuns &ru, const int32_t *tab, int m0, int n0) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < T::NX; ++i) {
      const int e = tid + 256 * i;
      if (XK) {
        xk[i] = e & (BK - 1);
        xr[i] = e >> 4;
      } else if (BLK) {
        xr[i] = (e & 15) + 16 * ((e >> 6) & (BM / 16 - 1));
        xk[i] = ((e >> 4) & 3) + 4 * (e >> (T::LM + 2));
      } else {
        xr[i] = e & (BM - 1);
        xk[i] = e >> T::LM;
      }
      xrow[i] = g_deposit((uint32_t)(m0 + xr[i]), ru.runsX, op.maskX) + (uint32_t)g_tab(tab, op.nS, xk[i]).x;
    }
#pragma unroll
    for (int i = 0; i < T::NY; ++i) {
      const int e = tid + 256 * i;
      if (YK) {
        yk[i] = e & (BK - 1);
        yn[i] = e >> 4;
      } else if (BLK) {
        yn[i] = (e & 15) + 16 * ((e >> 6) & (BN / 16 - 1));
        yk[i] = ((e >> 4) & 3) + 4 * (e >> (T::LN + 2));
      } else {
        yn[i] = e & (BN - 1);
        yk[i] = e >> T::LN;
      }
      ycol[i] = g_deposit((uint32_t)(n0 + yn[i]), ru.runsY, op.maskY) + (uint32_t)g_tab(tab, op.nS, yk[i]).y;
    }
  }
  __device__ __forceinline__ void fetch(const V *X, const V *Y, const DOp &op, const int32_t *tab, int k0) {
    const int2 t0 = g_tab(tab, op.nS, k0);
    const int bx = __builtin_amdgcn_readfirstlane(t0.x), by = __builtin_amdgcn_readfirstlane(t0.y);
#pragma unroll
    for (int i = 0; i < T::NX; ++i) xv[i] = X[xrow[i] + bx];
#pragma unroll
    for (int i = 0; i < T::NY; ++i) yv[i] = Y[by + ycol[i]];
  }
};

// Output tile `tile` of the op on one parameter vector's arena slice, 4M
// products in the precision of V (complex64: FP32, complex128: FP64).
// Summed entries [kb, ke) (multiples of 16); the tile is written to Z
// (row-major M x N).
template <typename V, bool XK, bool YK, int BM, int BN>
__device__ __forceinline__ void c4m_tile(V *__restrict__ As, V *__restrict__ Bs, const V *base, const DOp &op,
                                         const DRuns &ru, const int32_t *__restrict__ tab, int tile, int kb, int ke,
                                         V *__restrict__ Z) {
  using T = TileT<BM, BN>;
  using R = typename Acc4<V>::R;
  using A4 = typename Acc4<V>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a free index narrower than its tile side is one padded tile: rows /
  // columns past it read aliased operand entries and are not written
  const int sy = op.nFY > T::LN ? op.nFY - T::LN : 0;
  const int n0 = (tile & ((1 << sy) - 1)) * BN, m0 = (tile >> sy) * BM;
  const V *X = base + op.x;
  const V *Y = base + op.y;
  Stager<XK, YK, BM, BN, V> sg(op, ru, tab, m0, n0);
  A4 cre[T::WM][T::WN], cim[T::WM][T::WN];
#pragma unroll
  for (int i = 0; i < T::WM; ++i)
#pragma unroll
    for (int j = 0; j < T::WN; ++j) {
      cre[i][j] = A4{0, 0, 0, 0};
      cim[i][j] = A4{0, 0, 0, 0};
    }
  const int wr = (wave / T::GN) * 16 * T::WM, wc = (wave % T::GN) * 16 * T::WN;
  const int lr = lane & 15, lk = lane >> 4;  // MFMA operand row/col and real-k index
  const int part = lk & 1;

  sg.fetch(X, Y, op, tab, kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < T::NX; ++i) As[sg.xr[i] * T::AS + sg.xk[i]] = sg.xv[i];
#pragma unroll
    for (int i = 0; i < T::NY; ++i) Bs[sg.yk[i] * T::BS + sg.yn[i]] = sg.yv[i];
    __syncthreads();
    if (k0 + BK < ke) sg.fetch(X, Y, op, tab, k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kc = kk + (lk >> 1);
      R are[T::WM], aim[T::WM], bv[T::WN];
#pragma unroll
      for (int i = 0; i < T::WM; ++i) {
        const V x = As[(wr + 16 * i + lr) * T::AS + kc];
        are[i] = part ? -x.y : x.x;  // [Xr, -Xi]
        aim[i] = part ? x.x : x.y;   // [Xi,  Xr]
      }
#pragma unroll
      for (int j = 0; j < T::WN; ++j) {
        const V y = Bs[kc * T::BS + wc + 16 * j + lr];
        bv[j] = part ? y.y : y.x;  // [Yr; Yi]
      }
#pragma unroll
      for (int i = 0; i < T::WM; ++i)
#pragma unroll
        for (int j = 0; j < T::WN; ++j) {
          cre[i][j] = mfma4(are[i], bv[j], cre[i][j]);
          cim[i][j] = mfma4(aim[i], bv[j], cim[i][j]);
        }
    }
  }
  // result layout of the 16x16 tile (mfma4): column lane % 16, row per precision
  const int N = 1 << op.nFY, M = 1 << op.nFX;
#pragma unroll
  for (int i = 0; i < T::WM; ++i)
#pragma unroll
    for (int j = 0; j < T::WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * i + Acc4<V>::row(lk, r);
        const int col = n0 + wc + 16 * j + lr;
        if (row < M && col < N) Z[(int64_t)row * N + col] = make_c(cre[i][j][r], cim[i][j][r]);
      }
}

// --- split-BF16 products ----------------------------------------------------------------
// Every FP32 operand is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even); a product is taken as
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation
// (the lo*lo term, ~2^-16 relative, is dropped). Tiles hold packed
// (re, im) bf16 pairs; Re Z = (Xr, -Xi).(Yr, Yi) and Im Z = (Xr, Xi).(Yi, Yr)
// along the interleaved summed index, so one stage of 16 complex entries is
// one 32-deep MFMA per product.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

// (hi, lo) packed pairs of a complex value: low half re, high half im.
__device__ __forceinline__ void split_pack(float2 v, uint32_t &hi, uint32_t &lo) {
  const uint32_t hr = f2bf(v.x), hm = f2bf(v.y);
  const uint32_t lr = f2bf(v.x - bf2f(hr)), lm = f2bf(v.y - bf2f(hm));
  hi = hr | (hm << 16);
  lo = lr | (lm << 16);
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ u32x4 neg_im(u32x4 v) { return v ^ (u32x4){0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u}; }
__device__ __forceinline__ u32x4 swap_ri(u32x4 v) { return (v >> 16) | (v << 16); }

// LDS of the split-BF16 tile: X as [m][k] and Y as [n][k] (transposed)
// packed pairs, hi and lo parts.
template <bool XK, bool YK, int BM, int BN>
__device__ __forceinline__ void bf16x3_tile(uint32_t *__restrict__ Ah, uint32_t *__restrict__ Al,
                                            uint32_t *__restrict__ Bh, uint32_t *__restrict__ Bl, const float2 *base,
                                            const DOp &op, const DRuns &ru, const int32_t *__restrict__ tab, int tile,
                                            int kb, int ke, float2 *__restrict__ Z) {
  using T = TileT<BM, BN>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a free index narrower than its tile side is one padded tile: rows /
  // columns past it read aliased operand entries and are not written
  const int sy = op.nFY > T::LN ? op.nFY - T::LN : 0;
  const int n0 = (tile & ((1 << sy) - 1)) * BN, m0 = (tile >> sy) * BM;
  const float2 *X = base + op.x;
  const float2 *Y = base + op.y;
  Stager<XK, YK, BM, BN, float2, true> sg(op, ru, tab, m0, n0);
  mf4 cre[T::WM][T::WN], cim[T::WM][T::WN];
#pragma unroll
  for (int i = 0; i < T::WM; ++i)
#pragma unroll
    for (int j = 0; j < T::WN; ++j) {
      cre[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
    }
  const int wr = (wave / T::GN) * 16 * T::WM, wc = (wave % T::GN) * 16 * T::WN;
  const int lr = lane & 15, lg = lane >> 4;  // operand row/col, group of 4 complex summed entries

  sg.fetch(X, Y, op, tab, kb);
  for (int k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < T::NX; ++i) {
      uint32_t h, l;
      split_pack(sg.xv[i], h, l);
      Ah[sg.xr[i] * T::PS + sg.xk[i]] = h;
      Al[sg.xr[i] * T::PS + sg.xk[i]] = l;
    }
#pragma unroll
    for (int i = 0; i < T::NY; ++i) {
      uint32_t h, l;
      split_pack(sg.yv[i], h, l);
      Bh[sg.yn[i] * T::PS + sg.yk[i]] = h;
      Bl[sg.yn[i] * T::PS + sg.yk[i]] = l;
    }
    __syncthreads();
    if (k0 + BK < ke) sg.fetch(X, Y, op, tab, k0 + BK);
    u32x4 ah[T::WM], al[T::WM], bh[T::WN], bl[T::WN];
#pragma unroll
    for (int i = 0; i < T::WM; ++i) {
      ah[i] = *reinterpret_cast<const u32x4 *>(&Ah[(wr + 16 * i + lr) * T::PS + 4 * lg]);
      al[i] = *reinterpret_cast<const u32x4 *>(&Al[(wr + 16 * i + lr) * T::PS + 4 * lg]);
    }
#pragma unroll
    for (int j = 0; j < T::WN; ++j) {
      bh[j] = *reinterpret_cast<const u32x4 *>(&Bh[(wc + 16 * j + lr) * T::PS + 4 * lg]);
      bl[j] = *reinterpret_cast<const u32x4 *>(&Bl[(wc + 16 * j + lr) * T::PS + 4 * lg]);
    }
#pragma unroll
    for (int i = 0; i < T::WM; ++i) {
      const bf16x8 arh = as_bf(neg_im(ah[i])), arl = as_bf(neg_im(al[i]));
      const bf16x8 aih = as_bf(ah[i]), ail = as_bf(al[i]);
#pragma unroll
      for (int j = 0; j < T::WN; ++j) {
        const bf16x8 brh = as_bf(bh[j]), brl = as_bf(bl[j]);
        const bf16x8 bih = as_bf(swap_ri(bh[j])), bil = as_bf(swap_ri(bl[j]));
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brh, cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brl, cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, brh, cre[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bih, cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, bil, cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, bih, cim[i][j], 0, 0, 0);
      }
    }
  }
  const int N = 1 << op.nFY, M = 1 << op.nFX;
#pragma unroll
  for (int i = 0; i < T::WM; ++i)
#pragma unroll
    for (int j = 0; j < T::WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * i + 4 * lg + r;
        const int col = n0 + wc + 16 * j + lr;
        if (row < M && col < N) Z[(int64_t)row * N + col] = make_float2(cre[i][j][r], cim[i][j][r]);
      }
}

// One tile of any precision over summed entries [kb, ke), staged through
// the LDS at `lds` (kTileLds bytes, 16-byte aligned); base: the parameter
// vector's arena slice (complex128 for TN_MFMA_FP64, else complex64); z:
// where the M x N result goes.
template <int PREC, bool XK, bool YK, int BM, int BN>
__device__ __forceinline__ void any_tile(char *lds, const void *base, const DOp &op, const DRuns &ru,
                                         const int32_t *__restrict__ tab, int tile, int kb, int ke, void *z) {
  using T = TileT<BM, BN>;
  if constexpr (PREC == TN_MFMA_BF16X3) {
    uint32_t *Ah = reinterpret_cast<uint32_t *>(lds), *Al = Ah + BM * T::PS;
    uint32_t *Bh = Al + BM * T::PS, *Bl = Bh + BN * T::PS;
    bf16x3_tile<XK, YK, BM, BN>(Ah, Al, Bh, Bl, (const float2 *)base, op, ru, tab, tile, kb, ke, (float2 *)z);
  } else if constexpr (PREC == TN_MFMA_FP64) {
    double2 *As = reinterpret_cast<double2 *>(lds), *Bs = As + BM * T::AS;
    c4m_tile<double2, XK, YK, BM, BN>(As, Bs, (const double2 *)base, op, ru, tab, tile, kb, ke, (double2 *)z);
  } else {
    float2 *As = reinterpret_cast<float2 *>(lds), *Bs = As + BM * T::AS;
    c4m_tile<float2, XK, YK, BM, BN>(As, Bs, (const float2 *)base, op, ru, tab, tile, kb, ke, (float2 *)z);
  }
}

// LDS bytes of the largest tile of a precision (64 x 64).
template <int PREC>
constexpr int kTileLds = PREC == TN_MFMA_BF16X3 ? 4 * 64 * TileT<64, 64>::PS * 4
                         : PREC == TN_MFMA_FP64 ? (64 * TileT<64, 64>::AS + BK * TileT<64, 64>::BS) * 16
                                                : (64 * TileT<64, 64>::AS + BK * TileT<64, 64>::BS) * 8;

// Bytes of one complex element of a precision's operands.
constexpr int elem_bytes(int prec) { return prec == TN_MFMA_FP64 ? 16 : 8; }

}  // namespace

}  // namespace qtn
