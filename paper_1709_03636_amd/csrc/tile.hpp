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

// Staging assignment: each thread moves NX X and NY Y entries per stage.
// Summed-index offsets are sums over the set bits of k of one (X, Y) offset
// per summed bit (the offset table is built that way), so they are formed
// from those per-bit offsets, one bit per lane, read from the table once
// per tile: the offset of k0 + k (k0 a multiple of BK, k < BK) is the
// thread's fixed part t(k) plus the workgroup-uniform t(k0), formed in
// scalar registers, and no stage waits on a table read.
// XK: X's lowest address bit is summed (stage X with k fastest), else m
// fastest; YK likewise for Y. BLK (split-BF16 tiles, whose LDS rows are
// [row][k] with a 20-dword stride): with m (n) fastest, a wave stages a
// 16 x 4 block (16 consecutive rows, 128 contiguous bytes each, at 4 summed
// entries) instead of 64 rows at one summed entry, so its LDS writes fall
// on 64 different banks instead of 16.
// LDS element offsets: X entry (row m, summed k) at m * XM + k * XKS, Y
// entry (k, column n) at k * YKS + n * YN.
template <bool XK, bool YK, int BM, int BN, typename V, bool BLK, int XM, int XKS, int YKS, int YN>
struct Stager {
  using T = TileT<BM, BN>;
  int xs[T::NX], ys[T::NY];  // LDS offsets of this thread's entries
  uint32_t xrow[T::NX], ycol[T::NY];
  V xv[T::NX], yv[T::NY];
  int bx, by;  // lane t < nS: the X / Y offset of summed bit t
  // pk: null, or the bit positions of those offsets (each a power of two),
  // 5 bits per summed bit, six per word, X in pk[0..2] and Y in pk[3..5]:
  // no table read before the first stage's loads
  __device__ __forceinline__ Stager(const DOp &op, const DRuns &ru, const int32_t *tab, const int32_t *pk, int m0,
                                    int n0) {
    const int tid = threadIdx.x, lane = tid & 63;
    bx = by = 0;
    if (pk) {
      int w[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) w[i] = __builtin_amdgcn_readfirstlane(pk[i]);
      const int q = lane / 6, r = 5 * (lane - 6 * q);
      const int wx = q == 0 ? w[0] : q == 1 ? w[1] : w[2], wy = q == 0 ? w[3] : q == 1 ? w[4] : w[5];
      if (lane < op.nS) {
        bx = 1 << ((wx >> r) & 31);
        by = 1 << ((wy >> r) & 31);
      }
    } else if (lane < op.nS) {
      const int lo = op.nS < kTabLoBits ? op.nS : kTabLoBits;
      const int32_t *e = lane < kTabLoBits ? tab + (2 << lane) : tab + (2 << lo) + (2 << (lane - kTabLoBits));
      bx = e[0];
      by = e[1];
    }
    int lx[4], ly[4];  // offsets of summed bits 0-3 (zero past nS)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      lx[b] = __builtin_amdgcn_readlane(bx, b);
      ly[b] = __builtin_amdgcn_readlane(by, b);
    }
    auto low = [&](int k, const int *l) { return (k & 1 ? l[0] : 0) + (k & 2 ? l[1] : 0) + (k & 4 ? l[2] : 0) + (k & 8 ? l[3] : 0); };
#pragma unroll
    for (int i = 0; i < T::NX; ++i) {
      const int e = tid + 256 * i;
      int xr, xk;
      if (XK) {
        xk = e & (BK - 1);
        xr = e >> 4;
      } else if (BLK) {
        xr = (e & 15) + 16 * ((e >> 6) & (BM / 16 - 1));
        xk = ((e >> 4) & 3) + 4 * (e >> (T::LM + 2));
      } else {
        xr = e & (BM - 1);
        xk = e >> T::LM;
      }
      xs[i] = xr * XM + xk * XKS;
      xrow[i] = g_deposit((uint32_t)(m0 + xr), ru.runsX, op.maskX) + (uint32_t)low(xk, lx);
    }
#pragma unroll
    for (int i = 0; i < T::NY; ++i) {
      const int e = tid + 256 * i;
      int yk, yn;
      if (YK) {
        yk = e & (BK - 1);
        yn = e >> 4;
      } else if (BLK) {
        yn = (e & 15) + 16 * ((e >> 6) & (BN / 16 - 1));
        yk = ((e >> 4) & 3) + 4 * (e >> (T::LN + 2));
      } else {
        yn = e & (BN - 1);
        yk = e >> T::LN;
      }
      ys[i] = yk * YKS + yn * YN;
      ycol[i] = g_deposit((uint32_t)(n0 + yn), ru.runsY, op.maskY) + (uint32_t)low(yk, ly);
    }
  }
  // Stages are taken in Gray-code order over a power-of-two range of them,
  // so consecutive stages differ in one summed bit and the next stage's
  // offset is the current one plus or minus that bit's: stage s covers
  // summed entries kb + BK * (s ^ (s >> 1)). ox, oy: the offsets of the
  // stage fetched last.
  int ox, oy;
  __device__ __forceinline__ void load() {
#pragma unroll
    for (int i = 0; i < T::NX; ++i) xv[i] = X_[xrow[i] + ox];
#pragma unroll
    for (int i = 0; i < T::NY; ++i) yv[i] = Y_[oy + ycol[i]];
  }
  const V *X_, *Y_;
  // loads of stage 0 (summed entries from kb, a multiple of BK)
  __device__ __forceinline__ void first(const V *X, const V *Y, int kb) {
    X_ = X;
    Y_ = Y;
    ox = oy = 0;
    for (int t = 4; (kb >> t) != 0; ++t)
      if ((kb >> t) & 1) {
        ox += __builtin_amdgcn_readlane(bx, t);
        oy += __builtin_amdgcn_readlane(by, t);
      }
    load();
  }
  // loads of stage s >= 1: stage s - 1 with summed bit 4 + ctz(s) flipped
  __device__ __forceinline__ void next(int s) {
    const int b = __builtin_ctz((unsigned)s);
    const int dx = __builtin_amdgcn_readlane(bx, 4 + b), dy = __builtin_amdgcn_readlane(by, 4 + b);
    const bool set = ((s ^ (s >> 1)) >> b) & 1;
    ox += set ? dx : -dx;
    oy += set ? dy : -dy;
    load();
  }
};

// Output tile `tile` of the op on one parameter vector's arena slice, 4M
// products in the precision of V (complex64: FP32, complex128: FP64).
// Summed entries [kb, ke) (multiples of 16); the tile is written to Z
// (row-major M x N).
template <typename V, bool XK, bool YK, int BM, int BN>
__device__ __forceinline__ void c4m_tile(V *__restrict__ As, V *__restrict__ Bs, const V *base, const DOp &op,
                                         const DRuns &ru, const int32_t *__restrict__ tab, const int32_t *pk, int tile,
                                         int kb, int ke, V *__restrict__ Z) {
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
  Stager<XK, YK, BM, BN, V, false, T::AS, 1, T::BS, 1> sg(op, ru, tab, pk, m0, n0);
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

  const int S = (ke - kb) / BK;  // a power of two
  sg.first(X, Y, kb);
  for (int st = 0; st < S; ++st) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < T::NX; ++i) As[sg.xs[i]] = sg.xv[i];
#pragma unroll
    for (int i = 0; i < T::NY; ++i) Bs[sg.ys[i]] = sg.yv[i];
    __syncthreads();
    if (st + 1 < S) sg.next(st + 1);
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

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// (hi, lo) packed pairs of a complex value: low half re, high half im. The
// conversions round to nearest even (one v_cvt_pk_bf16_f32 per pair).
__device__ __forceinline__ void split_pack(float2 v, uint32_t &hi, uint32_t &lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v.x, v.y}, bf16x2));
  const float rr = v.x - __uint_as_float(hi << 16), ri = v.y - __uint_as_float(hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){rr, ri}, bf16x2));
}

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ u32x4 neg_im(u32x4 v) { return v ^ (u32x4){0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u}; }
__device__ __forceinline__ u32x4 swap_ri(u32x4 v) { return (v >> 16) | (v << 16); }

// LDS of the split-BF16 tile: X as [m][k] and Y as [n][k] (transposed)
// packed pairs, hi and lo parts. DB (one-item launches, whose workgroups
// have the LDS): two such buffers, stage s + 1 written into one while stage
// s is read from the other, one barrier per stage and the split of the next
// stage overlapping the matrix-core work of the current one; else one
// buffer and two barriers per stage.
template <bool XK, bool YK, int BM, int BN, bool DB>
__device__ __forceinline__ void bf16x3_tile(uint32_t *__restrict__ Ah, uint32_t *__restrict__ Al,
                                            uint32_t *__restrict__ Bh, uint32_t *__restrict__ Bl, const float2 *base,
                                            const DOp &op, const DRuns &ru, const int32_t *__restrict__ tab,
                                            const int32_t *pk, int tile, int kb, int ke, float2 *__restrict__ Z) {
  using T = TileT<BM, BN>;
  constexpr int BUF = (2 * BM + 2 * BN) * T::PS;  // words of one buffer (the four planes)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // a free index narrower than its tile side is one padded tile: rows /
  // columns past it read aliased operand entries and are not written
  const int sy = op.nFY > T::LN ? op.nFY - T::LN : 0;
  const int n0 = (tile & ((1 << sy) - 1)) * BN, m0 = (tile >> sy) * BM;
  const float2 *X = base + op.x;
  const float2 *Y = base + op.y;
  Stager<XK, YK, BM, BN, float2, true, T::PS, 1, 1, T::PS> sg(op, ru, tab, pk, m0, n0);
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

  // the staged stage (registers) split into buffer b
  auto write = [&](int b) {
#pragma unroll
    for (int i = 0; i < T::NX; ++i) {
      uint32_t h, l;
      split_pack(sg.xv[i], h, l);
      Ah[b * BUF + sg.xs[i]] = h;
      Al[b * BUF + sg.xs[i]] = l;
    }
#pragma unroll
    for (int i = 0; i < T::NY; ++i) {
      uint32_t h, l;
      split_pack(sg.yv[i], h, l);
      Bh[b * BUF + sg.ys[i]] = h;
      Bl[b * BUF + sg.ys[i]] = l;
    }
  };
  // the products of the stage in buffer b
  auto compute = [&](int b) {
    u32x4 ah[T::WM], al[T::WM], bh[T::WN], bl[T::WN];
#pragma unroll
    for (int i = 0; i < T::WM; ++i) {
      ah[i] = *reinterpret_cast<const u32x4 *>(&Ah[b * BUF + (wr + 16 * i + lr) * T::PS + 4 * lg]);
      al[i] = *reinterpret_cast<const u32x4 *>(&Al[b * BUF + (wr + 16 * i + lr) * T::PS + 4 * lg]);
    }
#pragma unroll
    for (int j = 0; j < T::WN; ++j) {
      bh[j] = *reinterpret_cast<const u32x4 *>(&Bh[b * BUF + (wc + 16 * j + lr) * T::PS + 4 * lg]);
      bl[j] = *reinterpret_cast<const u32x4 *>(&Bl[b * BUF + (wc + 16 * j + lr) * T::PS + 4 * lg]);
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
  };

  const int S = (ke - kb) / BK;  // a power of two
  sg.first(X, Y, kb);
  if constexpr (DB) {
    write(0);
    if (S > 1) sg.next(1);
    __syncthreads();
    for (int st = 0; st < S; ++st) {
      const int b = st & 1;
      compute(b);
      if (st + 1 < S) {
        write(b ^ 1);  // the other buffer's last readers passed the barrier that ended stage st - 1
        if (st + 2 < S) sg.next(st + 2);
      }
      __syncthreads();
    }
  } else {
    for (int st = 0; st < S; ++st) {
      __syncthreads();
      write(0);
      __syncthreads();
      if (st + 1 < S) sg.next(st + 1);
      compute(0);
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
// the LDS at `lds` (kTileLds bytes, 16-byte aligned; twice that with DB,
// which double-buffers the split-BF16 tile); pk: the packed summed-bit
// positions, or null for the offset table; base: the parameter
// vector's arena slice (complex128 for TN_MFMA_FP64, else complex64); z:
// where the M x N result goes.
template <int PREC, bool XK, bool YK, int BM, int BN, bool DB = false>
__device__ __forceinline__ void any_tile(char *lds, const void *base, const DOp &op, const DRuns &ru,
                                         const int32_t *__restrict__ tab, const int32_t *pk, int tile, int kb, int ke,
                                         void *z) {
  using T = TileT<BM, BN>;
  if constexpr (PREC == TN_MFMA_BF16X3) {
    uint32_t *Ah = reinterpret_cast<uint32_t *>(lds), *Al = Ah + BM * T::PS;
    uint32_t *Bh = Al + BM * T::PS, *Bl = Bh + BN * T::PS;
    bf16x3_tile<XK, YK, BM, BN, DB>(Ah, Al, Bh, Bl, (const float2 *)base, op, ru, tab, pk, tile, kb, ke, (float2 *)z);
  } else if constexpr (PREC == TN_MFMA_FP64) {
    double2 *As = reinterpret_cast<double2 *>(lds), *Bs = As + BM * T::AS;
    c4m_tile<double2, XK, YK, BM, BN>(As, Bs, (const double2 *)base, op, ru, tab, pk, tile, kb, ke, (double2 *)z);
  } else {
    float2 *As = reinterpret_cast<float2 *>(lds), *Bs = As + BM * T::AS;
    c4m_tile<float2, XK, YK, BM, BN>(As, Bs, (const float2 *)base, op, ru, tab, pk, tile, kb, ke, (float2 *)z);
  }
}

// LDS bytes of the largest tile of a precision (64 x 64).
template <int PREC>
constexpr int kTileLds = PREC == TN_MFMA_BF16X3 ? 4 * 64 * TileT<64, 64>::PS * 4
                         : PREC == TN_MFMA_FP64 ? (64 * TileT<64, 64>::AS + BK * TileT<64, 64>::BS) * 16
                                                : (64 * TileT<64, 64>::AS + BK * TileT<64, 64>::BS) * 8;

static_assert(kTileLds<TN_MFMA_BF16X3> == kTileLdsBytes<TN_MFMA_BF16X3> && kTileLds<TN_MFMA_FP32> == kTileLdsBytes<TN_MFMA_FP32> &&
                  kTileLds<TN_MFMA_FP64> == kTileLdsBytes<TN_MFMA_FP64>,
              "the planner's tile LDS sizes");

// Bytes of one complex element of a precision's operands.
constexpr int elem_bytes(int prec) { return prec == TN_MFMA_FP64 ? 16 : 8; }

}  // namespace

}  // namespace qtn
