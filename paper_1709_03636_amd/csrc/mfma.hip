// Pairwise contraction on the matrix cores (large steps of the level
// executor): eq. (1) as a complex GEMM
//   Z[m*N + n] = sum_k X[rX(m) + tX(k)] * Y[tY(k) + cY(n)],
// with rX / cY the deposit of the free-index bits into X / Y and (tX, tY)
// the op's summed-index offsets. The bit permutation is applied while the
// tiles are staged into LDS, so X and Y are read in their stored layout.
//
// Complex products use four real products (4M) on v_mfma_f32_16x16x4_f32
// with FP32 accumulation (or split-BF16 products, below): with the summed index interleaved as
// (re, im) pairs, Re Z = [Xr, -Xi] . [Yr; Yi] and Im Z = [Xi, Xr] . [Yr; Yi].
// Tile: 64 x 64 complex outputs per workgroup of four waves (32 x 32 each),
// 16 complex summed entries per LDS stage, next stage prefetched into
// registers while the matrix cores work on the current one.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace qtn {

typedef float mf4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int AS = BK + 1;  // LDS row stride of the X tile (float2), padded against bank conflicts
constexpr int BS = BN + 2;  // LDS row stride of the Y tile

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

__device__ __forceinline__ int2 g_tab(const int32_t *__restrict__ tb, int nS, int k) {
  if (nS <= kTabLoBits) return make_int2(tb[2 * k], tb[2 * k + 1]);
  const int lo = k & ((1 << kTabLoBits) - 1), hi = k >> kTabLoBits;
  const int32_t *h = tb + (2 << kTabLoBits);
  return make_int2(tb[2 * lo] + h[2 * hi], tb[2 * lo + 1] + h[2 * hi + 1]);
}

}  // namespace

// XK: X's lowest address bit is summed (stage X with k fastest), else m fastest.
// YK: Y's lowest address bit is summed (stage Y with k fastest), else n fastest.
template <bool XK, bool YK>
__global__ __launch_bounds__(256) void mfma_cgemm_kernel(LevelArgs a, DOp op, const int32_t *__restrict__ tab) {
  __shared__ float2 As[BM * AS];
  __shared__ float2 Bs[BK * BS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nT = 1 << (op.nFY - 6), mT = 1 << (op.nFX - 6);
  // XCD-aware tile order: consecutive workgroups land on different XCDs, so
  // give each XCD a contiguous run of tiles (shared X rows stay in its L2)
  const int nblk = nT * mT;
  int b = blockIdx.x;
  if (nblk % 8 == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int n0 = (b % nT) * BN, m0 = (b / nT) * BM;
  float2 *base = reinterpret_cast<float2 *>(a.arena) + (int64_t)blockIdx.z * a.stride;
  const float2 *X = base + op.x;
  const float2 *Y = base + op.y;
  float2 *Z = base + op.z;
  const int K = 1 << op.nS;

  // staging assignment: each thread moves 4 X and 4 Y entries per stage.
  // Summed-index offsets add over disjoint bits, so the offset of k0 + k
  // (k0 a multiple of BK, k < BK) is t(k0) + t(k): the per-thread parts
  // t(k) are fixed, and t(k0) is one workgroup-uniform lookup per stage.
  int xr[4], xk[4], yk[4], yn[4];
  uint32_t xrow[4], ycol[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i;
    if (XK) { xk[i] = e & (BK - 1); xr[i] = e >> 4; } else { xr[i] = e & (BM - 1); xk[i] = e >> 6; }
    if (YK) { yk[i] = e & (BK - 1); yn[i] = e >> 4; } else { yn[i] = e & (BN - 1); yk[i] = e >> 6; }
    xrow[i] = g_pdep((uint32_t)(m0 + xr[i]), op.maskX) + (uint32_t)g_tab(tab, op.nS, xk[i]).x;
    ycol[i] = g_pdep((uint32_t)(n0 + yn[i]), op.maskY) + (uint32_t)g_tab(tab, op.nS, yk[i]).y;
  }
  float2 xv[4], yv[4];
  auto fetch = [&](int k0) {
    const int2 t0 = g_tab(tab, op.nS, k0);
    const int bx = __builtin_amdgcn_readfirstlane(t0.x), by = __builtin_amdgcn_readfirstlane(t0.y);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xv[i] = X[xrow[i] + bx];
      yv[i] = Y[by + ycol[i]];
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      As[xr[i] * AS + xk[i]] = xv[i];
      Bs[yk[i] * BS + yn[i]] = yv[i];
    }
  };
  mf4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
    }
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;  // MFMA operand row/col and real-k index
  const int part = lk & 1;

  fetch(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BK < K) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kc = kk + (lk >> 1);
      float are[2], aim[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float2 x = As[(wr + 16 * i + lr) * AS + kc];
        are[i] = part ? -x.y : x.x;  // [Xr, -Xi]
        aim[i] = part ? x.x : x.y;   // [Xi,  Xr]
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float2 y = Bs[kc * BS + wc + 16 * j + lr];
        bv[j] = part ? y.y : y.x;  // [Yr; Yi]
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[i], bv[j], cre[i][j], 0, 0, 0);
          cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[i], bv[j], cim[i][j], 0, 0, 0);
        }
    }
  }
  // D layout of the 16x16 tile: lane holds rows 4*(lane/16)+r, column lane%16
  const int N = 1 << op.nFY;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * i + 4 * lk + r;
        const int col = n0 + wc + 16 * j + lr;
        Z[(int64_t)row * N + col] = make_float2(cre[i][j][r], cim[i][j][r]);
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

namespace {

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

constexpr int PS = BK + 4;  // packed-tile row stride (dwords), 16-byte aligned rows

}  // namespace

template <bool XK, bool YK>
__global__ __launch_bounds__(256) void mfma_cgemm_bf16x3_kernel(LevelArgs a, DOp op, const int32_t *__restrict__ tab) {
  __shared__ __align__(16) uint32_t Ah[BM * PS], Al[BM * PS];  // [m][k] packed pairs
  __shared__ __align__(16) uint32_t Bh[BN * PS], Bl[BN * PS];  // [n][k] (transposed) packed pairs
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nT = 1 << (op.nFY - 6), mT = 1 << (op.nFX - 6);
  const int nblk = nT * mT;
  int b = blockIdx.x;
  if (nblk % 8 == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
  const int n0 = (b % nT) * BN, m0 = (b / nT) * BM;
  float2 *base = reinterpret_cast<float2 *>(a.arena) + (int64_t)blockIdx.z * a.stride;
  const float2 *X = base + op.x;
  const float2 *Y = base + op.y;
  float2 *Z = base + op.z;
  const int K = 1 << op.nS;

  int xr[4], xk[4], yk[4], yn[4];
  uint32_t xrow[4], ycol[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i;
    if (XK) { xk[i] = e & (BK - 1); xr[i] = e >> 4; } else { xr[i] = e & (BM - 1); xk[i] = e >> 6; }
    if (YK) { yk[i] = e & (BK - 1); yn[i] = e >> 4; } else { yn[i] = e & (BN - 1); yk[i] = e >> 6; }
    xrow[i] = g_pdep((uint32_t)(m0 + xr[i]), op.maskX) + (uint32_t)g_tab(tab, op.nS, xk[i]).x;
    ycol[i] = g_pdep((uint32_t)(n0 + yn[i]), op.maskY) + (uint32_t)g_tab(tab, op.nS, yk[i]).y;
  }
  float2 xv[4], yv[4];
  auto fetch = [&](int k0) {
    const int2 t0 = g_tab(tab, op.nS, k0);
    const int bx = __builtin_amdgcn_readfirstlane(t0.x), by = __builtin_amdgcn_readfirstlane(t0.y);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xv[i] = X[xrow[i] + bx];
      yv[i] = Y[by + ycol[i]];
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t h, l;
      split_pack(xv[i], h, l);
      Ah[xr[i] * PS + xk[i]] = h;
      Al[xr[i] * PS + xk[i]] = l;
      split_pack(yv[i], h, l);
      Bh[yn[i] * PS + yk[i]] = h;
      Bl[yn[i] * PS + yk[i]] = l;
    }
  };

  mf4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
      cim[i][j] = mf4{0.f, 0.f, 0.f, 0.f};
    }
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lg = lane >> 4;  // operand row/col, group of 4 complex summed entries

  fetch(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + BK < K) fetch(k0 + BK);
    u32x4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const u32x4 *>(&Ah[(wr + 16 * i + lr) * PS + 4 * lg]);
      al[i] = *reinterpret_cast<const u32x4 *>(&Al[(wr + 16 * i + lr) * PS + 4 * lg]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      bh[j] = *reinterpret_cast<const u32x4 *>(&Bh[(wc + 16 * j + lr) * PS + 4 * lg]);
      bl[j] = *reinterpret_cast<const u32x4 *>(&Bl[(wc + 16 * j + lr) * PS + 4 * lg]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf16x8 arh = as_bf(neg_im(ah[i])), arl = as_bf(neg_im(al[i]));
      const bf16x8 aih = as_bf(ah[i]), ail = as_bf(al[i]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
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
  const int N = 1 << op.nFY;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr + 16 * i + 4 * lg + r;
        const int col = n0 + wc + 16 * j + lr;
        Z[(int64_t)row * N + col] = make_float2(cre[i][j][r], cim[i][j][r]);
      }
}

// True when the MFMA path takes this op (complex64, tiles divide the shape).
bool mfma_eligible(int dtype, const DOp &op) {
  return dtype == TN_C64 && op.type == OP_CONTRACT && op.nB == 0 && op.nFX >= 6 && op.nFY >= 6 && op.nS >= 4;
}

// prec: TN_MFMA_FP32 (4M FP32 products) or TN_MFMA_BF16X3 (split-BF16 products).
hipError_t mfma_contract(const LevelArgs &a, const DOp &op, const int32_t *tab, int prec, hipStream_t st) {
  const int nblk = 1 << (op.nFX - 6 + op.nFY - 6);
  dim3 grid(nblk, 1, a.n_sets);
  const bool xk = !(op.maskX & 1u), yk = !(op.maskY & 1u);
  if (prec == TN_MFMA_BF16X3) {
    if (xk && yk) hipLaunchKernelGGL((mfma_cgemm_bf16x3_kernel<true, true>), grid, dim3(256), 0, st, a, op, tab);
    else if (xk) hipLaunchKernelGGL((mfma_cgemm_bf16x3_kernel<true, false>), grid, dim3(256), 0, st, a, op, tab);
    else if (yk) hipLaunchKernelGGL((mfma_cgemm_bf16x3_kernel<false, true>), grid, dim3(256), 0, st, a, op, tab);
    else hipLaunchKernelGGL((mfma_cgemm_bf16x3_kernel<false, false>), grid, dim3(256), 0, st, a, op, tab);
    return hipGetLastError();
  }
  if (xk && yk) hipLaunchKernelGGL((mfma_cgemm_kernel<true, true>), grid, dim3(256), 0, st, a, op, tab);
  else if (xk) hipLaunchKernelGGL((mfma_cgemm_kernel<true, false>), grid, dim3(256), 0, st, a, op, tab);
  else if (yk) hipLaunchKernelGGL((mfma_cgemm_kernel<false, true>), grid, dim3(256), 0, st, a, op, tab);
  else hipLaunchKernelGGL((mfma_cgemm_kernel<false, false>), grid, dim3(256), 0, st, a, op, tab);
  return hipGetLastError();
}

}  // namespace qtn
