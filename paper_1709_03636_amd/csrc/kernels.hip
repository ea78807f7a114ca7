// HIP kernels for gfx950: angle binding, the fused per-workgroup network
// executor (forward and adjoint), and the FP64 objective combine.
//
// Fused executor: one workgroup runs one (network, parameter vector) task at
// a time (persistent grid, contiguous runs of tasks sorted by cost). All
// tensors of the task live in LDS: constant leaves and the parametric leaves
// bound for its parameter vector are copied in, and every pairwise
// contraction (eq. (1))
// reads its operands through per-op address maps and writes its result into
// the LDS arena. Rank-0 results (the last contraction of each component)
// are accumulated in FP64 with a fixed reduction tree, so results are
// deterministic.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"
#include "kargs.hpp"
#include "lrec.hpp"

namespace qtn {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename V> __device__ __forceinline__ V from_d2(double2 v);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }

// Read-only data read with workgroup-uniform addresses (op descriptors,
// offset tables) goes through the constant address space so the compiler
// can use scalar loads for it. Nothing the kernels write is read this way.
#define QTN_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const QTN_CONST T *cptr(const T *p) {
  return (const QTN_CONST T *)(p);
}
// Word-wise load of a descriptor struct through the constant address space.
template <typename S>
__device__ __forceinline__ S cload(const S *p) {
  static_assert(sizeof(S) % 4 == 0, "descriptor size");
  S r;
  const QTN_CONST int32_t *src = (const QTN_CONST int32_t *)(p);
  int32_t *dst = reinterpret_cast<int32_t *>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) dst[i] = src[i];
  return r;
}

// (X, Y) offsets of summed index k from an op's table (low/high split
// beyond kTabLoBits summed bits).
__device__ __forceinline__ int2 tab_at(const int32_t *__restrict__ tb, int nS, int k) {
  if (nS <= kTabLoBits) return make_int2(tb[2 * k], tb[2 * k + 1]);
  const int lo = k & ((1 << kTabLoBits) - 1), hi = k >> kTabLoBits;
  const int32_t *h = tb + (2 << kTabLoBits);
  return make_int2(tb[2 * lo] + h[2 * hi], tb[2 * lo + 1] + h[2 * hi + 1]);
}

// Deposit the low bits of v at the set positions of mask (lowest first).
__device__ __forceinline__ uint32_t pdep32(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    uint32_t low = mask & (0u - mask);
    if (v & 1u) r |= low;
    v >>= 1;
    mask ^= low;
  }
  return r;
}

// Operand offsets (X, Y) of output c of an op (see DOp: c = (i, b, j)).
__device__ __forceinline__ void out_addr(const DOp &op, const int32_t *__restrict__ tbB, uint32_t c, uint32_t &fx,
                                         uint32_t &fy) {
  const uint32_t rest = c >> op.nFY;
  fy = pdep32(c & ((1u << op.nFY) - 1u), op.maskY);
  fx = pdep32(rest >> op.nB, op.maskX);
  if (op.nB) {
    const uint32_t b = rest & ((1u << op.nB) - 1u);
    fx += tbB[2 * b];
    fy += tbB[2 * b + 1];
  }
}

// --- parametric tensors ---------------------------------------------------------
// U(theta) = exp(-i theta P / 2) = c I - i s P with c = cos(theta/2),
// s = sin(theta/2); dU/dtheta has the same form with (c, s) -> (-s/2, c/2).

// Entry (r, col) of the Pauli (product) of a parametric gate kind.
__device__ __forceinline__ double2 pauli_rc(int kind, int r, int col) {
  if (kind == TN_RX) return make_double2(r != col ? 1.0 : 0.0, 0.0);
  if (kind == TN_RY) return make_double2(0.0, r == col ? 0.0 : (r == 0 ? -1.0 : 1.0));
  if (kind == TN_RZ) return make_double2(r == col ? (r == 0 ? 1.0 : -1.0) : 0.0, 0.0);
  // Z(x)Z = diag(1, -1, -1, 1): sign is the parity of the two bits
  return make_double2(r == col ? (((r ^ (r >> 1)) & 1) ? -1.0 : 1.0) : 0.0, 0.0);
}

__device__ __forceinline__ double2 u_rc(int kind, int r, int col, double c, double s) {
  double2 p = pauli_rc(kind, r, col);
  // c*delta - i*s*(p.x + i p.y) = (c*delta + s*p.y) + i(-s*p.x)
  return make_double2((r == col ? c : 0.0) + s * p.y, -s * p.x);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// Entry `idx` (canonical wire order) of the tensor of a parametric gate:
// unfolded U, or folded U (x) conj(U) with wires (out..., in...), each wire
// (ket bit, bra bit). deriv selects d/dtheta.
__device__ double2 param_entry(int kind, int folded, int idx, double c, double s, bool deriv) {
  const int nq = kind == TN_ZZ ? 2 : 1;
  const double dc = -0.5 * s, ds = 0.5 * c;
  if (!folded) {
    int r = idx >> nq, col = idx & ((1 << nq) - 1);
    return deriv ? u_rc(kind, r, col, dc, ds) : u_rc(kind, r, col, c, s);
  }
  int rk, rb, ck, cb;  // ket row, bra row, ket col, bra col
  if (nq == 1) {
    rk = (idx >> 3) & 1; rb = (idx >> 2) & 1; ck = (idx >> 1) & 1; cb = idx & 1;
  } else {
    int a0 = (idx >> 7) & 1, b0 = (idx >> 6) & 1, a1 = (idx >> 5) & 1, b1 = (idx >> 4) & 1;
    int c0 = (idx >> 3) & 1, d0 = (idx >> 2) & 1, c1 = (idx >> 1) & 1, d1 = idx & 1;
    rk = 2 * a0 + a1; rb = 2 * b0 + b1; ck = 2 * c0 + c1; cb = 2 * d0 + d1;
  }
  double2 uk = u_rc(kind, rk, ck, c, s), ub = conj2(u_rc(kind, rb, cb, c, s));
  if (!deriv) return cmul(uk, ub);
  double2 duk = u_rc(kind, rk, ck, dc, ds), dub = conj2(u_rc(kind, rb, cb, dc, ds));
  double2 t1 = cmul(duk, ub), t2 = cmul(uk, dub);
  return make_double2(t1.x + t2.x, t1.y + t2.y);
}

// Angle binding (one workgroup per parametric tensor and parameter vector):
// G[s][off + e] = entry e of the tensor at angle coeff * params[s][param], and
// optionally dG[s][off + e] = its derivative with respect to that angle.
template <typename V>
__global__ __launch_bounds__(256) void bind_params_kernel(const DParam *__restrict__ slots,
                                                          const double *__restrict__ params, int n_params,
                                                          int per_set, V *__restrict__ G, V *__restrict__ dG) {
  const int s = blockIdx.y;
  const DParam d = slots[blockIdx.x];
  const double th = d.coeff * params[(size_t)s * n_params + d.param];
  double sn, cs;
  sincos(0.5 * th, &sn, &cs);
  V *g = G + (size_t)s * per_set + d.off;
  V *dg = dG ? dG + (size_t)s * per_set + d.off : nullptr;
  // a diagonal tensor holds entries (e, e) of the full one: index e (2^bits + 1)
  const int stride = d.diag ? (1 << d.bits) + 1 : 1;
  for (int e = threadIdx.x; e < (1 << d.bits); e += blockDim.x) {
    g[e] = from_d2<V>(param_entry(d.kind, d.folded, e * stride, cs, sn, false));
    if (dg) dg[e] = from_d2<V>(param_entry(d.kind, d.folded, e * stride, cs, sn, true));
  }
}

// Sum over the wave, returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum_f64(v, 6);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// Fixed-tree block sum; the result is valid in thread 0. red: BLOCK/64 doubles.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  if (BLOCK == 64) return v;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BLOCK / 64; ++i) r += red[i];
  __syncthreads();
  return r;
}

// --- reductions -------------------------------------------------------------------
// (cross-lane group sums: lrec.hpp)

// --- fused executor ------------------------------------------------------------------

// Contraction with a compile-time number of summed entries K = 2^LGK: the
// op's offset table (2K ints, uniform across the workgroup) is held in
// scalar registers and the K loop is unrolled, so all operand reads of an
// output are in flight together. One output per lane.
template <typename V, int BLOCK, int LGK>
__device__ __forceinline__ void contract_small_k(V *mem, const DOp &op, const int32_t *__restrict__ tb,
                                                 const int32_t *__restrict__ tbB) {
  constexpr int K = 1 << LGK;
  int32_t t[2 * K];
  const QTN_CONST int32_t *tc = cptr(tb);
#pragma unroll
  for (int i = 0; i < 2 * K; ++i) t[i] = tc[i];
  const int nOut = 1 << (op.nFX + op.nB + op.nFY);
  const V *X = mem + op.x;
  const V *Y = mem + op.y;
  V *Z = mem + op.z;
  for (int c = threadIdx.x; c < nOut; c += BLOCK) {
    uint32_t fx, fy;
    out_addr(op, tbB, (uint32_t)c, fx, fy);
    // operand reads in chunks of up to 8 entries, all issued before the
    // multiply-adds that consume them
    constexpr int CH = K < 8 ? K : 8;
    V acc = czero<V>();
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += CH) {
      V xv[CH], yv[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        xv[k] = X[fx + t[2 * (k0 + k)]];
        yv[k] = Y[fy + t[2 * (k0 + k) + 1]];
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) acc = cmul_add(acc, xv[k], yv[k]);
    }
    Z[c] = acc;
  }
}

// General contraction (any K); with fewer outputs than lanes the summed
// index is split over lane groups and the partial sums are added in a fixed
// order through `scratch`.
template <typename V, int BLOCK>
__device__ __forceinline__ void contract_general(V *mem, const DOp &op, const int32_t *__restrict__ tb,
                                                 const int32_t *__restrict__ tbB, V *scratch) {
  const int tid = threadIdx.x;
  const int lgOut = op.nFX + op.nB + op.nFY;
  const int nOut = 1 << lgOut;
  const int K = 1 << op.nS;
  const V *X = mem + op.x;
  const V *Y = mem + op.y;
  V *Z = mem + op.z;
  if (nOut >= BLOCK) {
    for (int c = tid; c < nOut; c += BLOCK) {
      uint32_t fx, fy;
      out_addr(op, tbB, (uint32_t)c, fx, fy);
      V acc = czero<V>();
      for (int k = 0; k < K; ++k) {
        const int2 o = tab_at(tb, op.nS, k);
        acc = cmul_add(acc, X[fx + o.x], Y[fy + o.y]);
      }
      Z[c] = acc;
    }
  } else {
    int lgG = 0;
    while ((nOut << (lgG + 1)) <= BLOCK && lgG < op.nS) ++lgG;
    const int G = 1 << lgG;
    const int c = tid & (nOut - 1);
    const int g = tid >> lgOut;
    if (g < G) {
      uint32_t fx, fy;
      out_addr(op, tbB, (uint32_t)c, fx, fy);
      V acc = czero<V>();
      for (int k = g; k < K; k += G) {
        const int2 o = tab_at(tb, op.nS, k);
        acc = cmul_add(acc, X[fx + o.x], Y[fy + o.y]);
      }
      scratch[tid] = acc;
    }
    __syncthreads();
    if (tid < nOut) {
      V s = scratch[tid];
      for (int gg = 1; gg < G; ++gg) s = cadd(s, scratch[gg * nOut + tid]);
      Z[tid] = s;
    }
  }
}

template <typename V, int BLOCK>
__device__ __forceinline__ void op_contract(V *mem, const DOp &op, const int32_t *__restrict__ tb,
                                            const int32_t *__restrict__ tbB, V *scratch) {
  switch (op.nS) {
    case 0: contract_small_k<V, BLOCK, 0>(mem, op, tb, tbB); break;
    case 1: contract_small_k<V, BLOCK, 1>(mem, op, tb, tbB); break;
    case 2: contract_small_k<V, BLOCK, 2>(mem, op, tb, tbB); break;
    case 3: contract_small_k<V, BLOCK, 3>(mem, op, tb, tbB); break;
    case 4: contract_small_k<V, BLOCK, 4>(mem, op, tb, tbB); break;
    default: contract_general<V, BLOCK>(mem, op, tb, tbB, scratch); break;
  }
}

// Rank-0 contraction from a lane record, in FP64.
template <typename V>
__device__ __forceinline__ void scalar_rec(const V *mem, double2 *scal, const int4 &rec, uint32_t hdr) {
  const int K = 1 << ((hdr >> 3) & 15u);
  double re = 0.0, im = 0.0;
  if ((int)threadIdx.x < K) {
    const double2 x = to_d2(mem[rec.x]);
    const double2 y = to_d2(mem[rec.y]);
    re = x.x * y.x - x.y * y.y;
    im = x.x * y.y + x.y * y.x;
  }
  const double2 v = group_sum(make_double2(re, im), 6);
  if (threadIdx.x == 63) scal[hdr >> 15] = v;
}

// Fused executor. GRAD selects the forward+adjoint program: the adjoint of
// each parametric leaf is contracted with the leaf's angle derivative (bound
// by the binding kernel) as soon as it is formed, and summed per parameter in
// FP64. RONLY (64-lane workgroups): every op has a lane record, the
// descriptor path is left out. GMEM: the network's memory is not LDS but the
// workgroup's slot of a global arena (networks too large for LDS whose
// steps are still small: no launch per step, the slot stays in L2/MALL);
// scratch, scalars and gradient sums stay in LDS.
template <typename T, int BLOCK, bool GRAD, bool RONLY, bool GMEM>
__global__ __launch_bounds__(BLOCK) void fused_exec_kernel(FusedArgs a) {
  using V = typename Cplx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  V *mem = GMEM ? reinterpret_cast<V *>(a.garena) + (size_t)blockIdx.x * a.garena_stride : reinterpret_cast<V *>(smem);
  V *scratch = reinterpret_cast<V *>(smem + a.scratch_off);
  double2 *scal = reinterpret_cast<double2 *>(smem + a.scal_off);
  double *gacc = reinterpret_cast<double *>(smem + a.gacc_off);
  double *red = reinterpret_cast<double *>(smem + a.red_off);
  const int tid = threadIdx.x;
  const V *consts = reinterpret_cast<const V *>(a.consts);
  const V *bound = reinterpret_cast<const V *>(a.bound);
  const V *dbound = reinterpret_cast<const V *>(a.dbound);

  // tasks are ordered by decreasing network cost, network-major; workgroup b
  // takes a contiguous run, so its consecutive tasks mostly share one program
  const int t_end = min(a.n_tasks, ((int)blockIdx.x + 1) * a.per_block);
  for (int task = blockIdx.x * a.per_block; task < t_end; ++task) {
    const int ni = cptr(a.task_net)[task / a.n_sets];
    const int set = task % a.n_sets;
    const DNet net = cload(a.nets + ni);

    for (int e = tid; e < net.n_const; e += BLOCK) mem[e] = consts[net.const_begin + e];
    const V *bset = bound + (size_t)set * a.per_set;
    for (int t = 0; t < net.n_ptens; ++t) {
      const DParam d = cload(a.ptens + net.ptens_begin + t);
      for (int e = tid; e < (1 << d.bits); e += BLOCK) mem[d.off + e] = bset[d.slot + e];
    }
    if (GRAD)
      for (int p = tid; p < a.n_params; p += BLOCK) gacc[p] = 0.0;
    __syncthreads();

    // Descriptors are read when needed, not prefetched: scalar and LDS
    // loads share one wait counter, so an outstanding descriptor load would
    // delay every LDS wait of the current op.
    const DOp *ops = a.ops + net.op_begin;
    // lane records (64-lane workgroups): the records of the next two ops are
    // in flight while the current op runs (vector loads: their wait counter
    // is not the LDS one; two hide an L2 hit, more cost occupancy)
    const int4 *recs = a.recs + (size_t)net.rec_begin * kRecLanes + (tid & (kRecLanes - 1));
    int4 rec = make_int4(0, 0, 0, 0);
    int4 rec1 = make_int4(0, 0, 0, 0);
    if (BLOCK == kRecLanes && net.n_ops > 0) rec = recs[0];
    if (BLOCK == kRecLanes && net.n_ops > 1) rec1 = recs[kRecLanes];
    for (int o = 0; o < net.n_ops; ++o) {
      int4 nrec = make_int4(0, 0, 0, 0);
      if (BLOCK == kRecLanes) {
        if (o + 2 < net.n_ops) nrec = recs[(size_t)(o + 2) * kRecLanes];
        const uint32_t hdr = (uint32_t)__builtin_amdgcn_readfirstlane(rec.w);
        const uint32_t type = hdr & 7u;
        if (type == kRecLite) {
          switch ((hdr >> 3) & 15u) {
            case 0: contract_lite<V, 0>(mem, rec, hdr); break;
            case 1: contract_lite<V, 1>(mem, rec, hdr); break;
            default: contract_lite<V, 2>(mem, rec, hdr); break;
          }
        } else if (type == kRecWide) {
          contract_wide<V>(mem, rec, hdr);
        } else if (type == kRecNarrow) {
          contract_narrow<V>(mem, rec, hdr);
        } else if (type == kRecScalar) {
          scalar_rec<V>(mem, scal, rec, hdr);
        } else if (GRAD && type == kRecSeed) {
          if (tid == 0) {
            const int skip = rec.x;
            double2 p = make_double2(1.0, 0.0);
            for (int j = 0; j < net.n_comp; ++j)
              if (j != skip) p = cmul(p, scal[j]);
            mem[hdr >> 15] = from_d2<V>(p);
          }
        } else if (GRAD && type == kRecLeafGrad) {
          // entries l + 64 q: adjoint times the bound angle derivative
          const int cnt = 1 << ((hdr >> 7) & 15u);
          const int slot = __builtin_amdgcn_readlane(rec.z, 0);
          const uint32_t clo = (uint32_t)__builtin_amdgcn_readlane(rec.z, 1);
          const uint32_t chi = (uint32_t)__builtin_amdgcn_readlane(rec.z, 2);
          const double coeff = __hiloint2double((int)chi, (int)clo);
          const V *dv = dbound + (size_t)set * a.per_set + slot;
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (tid + 64 * q < cnt) {
              const double2 g = to_d2(mem[rec.x + 64 * q]);
              const double2 w = to_d2(dv[((uint32_t)rec.y >> (8 * q)) & 0xffu]);
              acc += g.x * w.x - g.y * w.y;
            }
          acc = group_sum_f64(acc, 6);
          if (tid == 63) gacc[hdr >> 15] += coeff * acc;
        }
        if (RONLY || type != 0) {
          __syncthreads();
          rec = rec1;
          rec1 = nrec;
          continue;
        }
      }
      const DOp op = cload(ops + o);
      const int32_t *tb = a.tabs + op.tab;
      if (op.type == OP_CONTRACT) {
        op_contract<V, BLOCK>(mem, op, tb, a.tabs + op.tabB, scratch);
      } else if (op.type == OP_SCALAR) {
        const int K = 1 << op.nS;
        double re = 0.0, im = 0.0;
        for (int k = tid; k < K; k += BLOCK) {
          const int2 o = tab_at(tb, op.nS, k);
          const double2 x = to_d2(mem[op.x + o.x]);
          const double2 y = to_d2(mem[op.y + o.y]);
          re += x.x * y.x - x.y * y.y;
          im += x.x * y.y + x.y * y.x;
        }
        re = block_sum<BLOCK>(re, red);
        im = block_sum<BLOCK>(im, red);
        if (tid == 0) scal[op.z] = make_double2(re, im);
      } else if (GRAD && op.type == OP_SEED) {
        if (tid == 0) {
          double2 p = make_double2(1.0, 0.0);
          for (int j = 0; j < net.n_comp; ++j)
            if (j != op.aux0) p = cmul(p, scal[j]);
          mem[op.z] = from_d2<V>(p);
        }
      } else if (GRAD) {  // OP_LEAFGRAD: theta-derivative of the leaf, contracted with its adjoint
        const DParam d = cload(a.ptens + op.aux0);
        const V *dv = dbound + (size_t)set * a.per_set + d.slot;
        double acc = 0.0;
        for (int i = tid; i < (1 << op.nFX); i += BLOCK) {
          const double2 g = to_d2(mem[op.x + i]);
          const double2 w = to_d2(dv[tb[i]]);
          acc += g.x * w.x - g.y * w.y;
        }
        acc = block_sum<BLOCK>(acc, red);
        if (tid == 0) gacc[d.param] += d.coeff * acc;
      }
      __syncthreads();
      rec = rec1;
      rec1 = nrec;
    }

    if (tid == 0) {
      double2 p = make_double2(1.0, 0.0);
      for (int j = 0; j < net.n_comp; ++j) p = cmul(p, scal[j]);
      double *ov = a.out_val + ((size_t)ni * a.n_sets + set) * 2;
      ov[0] = p.x;
      ov[1] = p.y;
    }
    if (GRAD)
      for (int p = tid; p < a.n_params; p += BLOCK) a.out_grad[((size_t)ni * a.n_sets + set) * a.n_params + p] = gacc[p];
    __syncthreads();
  }
}

// --- set-packed fused executor ----------------------------------------------------------
// One 64-lane wave runs S = 2 or 4 angle sets of one network: lane
// l = s * W + w (W = 64 / S) serves set s. Small steps (4 to 16 products per
// set) then fill the wave instead of leaving most lanes idle, and the
// per-op decode is shared by the sets.

__device__ __forceinline__ int2 unpack16(uint32_t t) { return make_int2((int)(t & 0xffffu), (int)(t >> 16)); }

// kSetContract (see device.hpp); 2^LGW lanes per set.
template <typename V, int LGW>
__device__ __forceinline__ void set_contract(V *m, const int4 &rec, uint32_t hdr, int w) {
  const int lgG = (hdr >> 3) & 7, lgQ = (hdr >> 6) & 7, lgR = (hdr >> 9) & 7, lgOut = (hdr >> 12) & 15;
  const int z = (int)(hdr >> 16);
  const int R = 1 << lgR;
  if (lgQ == 0) {
    V acc = czero<V>();
    for (int i = 0; i < R; i += 4) {
      V xv[4], yv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i + u < R) {
          const int2 t = unpack16((uint32_t)__builtin_amdgcn_readlane(rec.z, i + u));
          xv[u] = m[rec.x + t.x];
          yv[u] = m[rec.y + t.y];
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i + u < R) acc = cmul_add(acc, xv[u], yv[u]);
    }
    acc = group_sum(acc, lgG);
    const int j = w >> lgG;
    if ((w & ((1 << lgG) - 1)) == 0 && j < (1 << lgOut)) m[z + j] = acc;
  } else {  // G = 1: outputs w + W q, four at a time
    const int Q = 1 << lgQ;
    for (int q0 = 0; q0 < Q; q0 += 4) {
      int2 d[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        d[u] = (q0 + u == 0 || q0 + u >= Q) ? make_int2(0, 0)
                                            : unpack16((uint32_t)__builtin_amdgcn_readlane(rec.w, q0 + u));
      V acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = czero<V>();
      for (int i = 0; i < R; ++i) {
        const int2 t = unpack16((uint32_t)__builtin_amdgcn_readlane(rec.z, i));
        V xv[4], yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u < Q) {
            xv[u] = m[rec.x + d[u].x + t.x];
            yv[u] = m[rec.y + d[u].y + t.y];
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u < Q) acc[u] = cmul_add(acc[u], xv[u], yv[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + u < Q) m[z + w + ((q0 + u) << LGW)] = acc[u];
    }
  }
}

// kSetScalar: FP64 products and sums.
template <typename V>
__device__ __forceinline__ void set_scalar(const V *m, double2 *scal, const int4 &rec, uint32_t hdr, int w) {
  const int lgG = (hdr >> 3) & 7, lgR = (hdr >> 9) & 7;
  const int R = 1 << lgR;
  double2 acc = make_double2(0.0, 0.0);
  for (int i = 0; i < R; ++i) {
    const int2 t = unpack16((uint32_t)__builtin_amdgcn_readlane(rec.z, i));
    const double2 x = to_d2(m[rec.x + t.x]);
    const double2 y = to_d2(m[rec.y + t.y]);
    acc.x += x.x * y.x - x.y * y.y;
    acc.y += x.x * y.y + x.y * y.x;
  }
  acc = group_sum(acc, lgG);
  if (w == 0) scal[hdr >> 16] = acc;
}

// kSetLeafGrad: Re(sum_e adjoint[e] * dU[index(e)]) in FP64, added to the
// parameter's accumulator.
template <typename V>
__device__ __forceinline__ void set_leafgrad(const V *m, const V *dv, double *gacc, const int4 &rec, uint32_t hdr,
                                             int w) {
  const int lgG = (hdr >> 3) & 7, lgR = (hdr >> 9) & 7;
  const int R = 1 << lgR;
  const int slot = __builtin_amdgcn_readlane(rec.w, 1);
  const double coeff = __hiloint2double(__builtin_amdgcn_readlane(rec.w, 3), __builtin_amdgcn_readlane(rec.w, 2));
  dv += slot;
  double acc = 0.0;
  constexpr int U = 4;
  for (int i = 0; i < R; i += U) {
    V gv[U], dvv[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u < R) {
        const int t = __builtin_amdgcn_readlane(rec.z, i + u);
        gv[u] = m[rec.x + ((i + u) << lgG)];
        dvv[u] = dv[rec.y + t];
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u < R) {
        const double2 g = to_d2(gv[u]), d = to_d2(dvv[u]);
        acc += g.x * d.x - g.y * d.y;
      }
  }
  acc = group_sum_f64(acc, lgG);
  if (w == 0) gacc[hdr >> 16] += coeff * acc;
}

// n elements src -> dst by the W lanes of one set, four loads in flight.
template <typename V, int W>
__device__ __forceinline__ void set_copy(V *dst, const V *src, int n, int w) {
  int e = w;
  for (; e + 3 * W < n; e += 4 * W) {
    const V a0 = src[e], a1 = src[e + W], a2 = src[e + 2 * W], a3 = src[e + 3 * W];
    dst[e] = a0;
    dst[e + W] = a1;
    dst[e + 2 * W] = a2;
    dst[e + 3 * W] = a3;
  }
  for (; e < n; e += W) dst[e] = src[e];
}

// Set-packed fused executor: a task is (network, group of 64 / 2^LGW angle
// sets, 2^LGW lanes each); every op of every program has a set-packed
// record. Sets past n_sets in the last group recompute the last set and
// write nothing.
template <typename T, bool GRAD, int LGW>
__global__ __launch_bounds__(64) void fused_sets_kernel(FusedArgs a) {
  using V = typename Cplx<T>::type;
  constexpr int W = 1 << LGW, S = 64 >> LGW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x, s = lane >> LGW, w = lane & (W - 1);
  V *m = reinterpret_cast<V *>(smem) + (size_t)s * a.set_stride;
  double2 *scal = reinterpret_cast<double2 *>(smem + a.scal_off) + s * a.max_comp;
  double *gacc = reinterpret_cast<double *>(smem + a.gacc_off) + s * a.n_params;
  const V *consts = reinterpret_cast<const V *>(a.consts);
  const V *bound = reinterpret_cast<const V *>(a.bound);
  const V *dbound = reinterpret_cast<const V *>(a.dbound);

  const int t_end = min(a.n_tasks, ((int)blockIdx.x + 1) * a.per_block);
  for (int task = blockIdx.x * a.per_block; task < t_end; ++task) {
    const int ni = cptr(a.task_net)[task / a.n_groups];
    const int set = (task % a.n_groups) * S + s;
    const bool valid = set < a.n_sets;
    const int setc = valid ? set : a.n_sets - 1;
    const DNet net = cload(a.nets + ni);

    set_copy<V, W>(m, consts + net.const_begin, net.n_const, w);
    const V *bset = bound + (size_t)setc * a.per_set;
    for (int t = 0; t < net.n_ptens; ++t) {
      const DParam d = cload(a.ptens + net.ptens_begin + t);
      set_copy<V, W>(m + d.off, bset + d.slot, 1 << d.bits, w);
    }
    if (GRAD)
      for (int p = w; p < a.n_params; p += W) gacc[p] = 0.0;
    __syncthreads();

    const V *dv = dbound + (size_t)setc * a.per_set;
    const int4 *recs = a.recs + (size_t)net.rec_begin * W + w;
    int4 rec = make_int4(0, 0, 0, 0), rec1 = make_int4(0, 0, 0, 0);
    if (net.n_ops > 0) rec = recs[0];
    if (net.n_ops > 1) rec1 = recs[W];
    for (int o = 0; o < net.n_ops; ++o) {
      int4 nrec = make_int4(0, 0, 0, 0);
      if (o + 2 < net.n_ops) nrec = recs[(size_t)(o + 2) * W];
      const uint32_t hdr = (uint32_t)__builtin_amdgcn_readfirstlane(rec.w);
      const uint32_t type = hdr & 7u;
      if (type == kSetContract) {
        set_contract<V, LGW>(m, rec, hdr, w);
      } else if (type == kSetScalar) {
        set_scalar<V>(m, scal, rec, hdr, w);
      } else if (GRAD && type == kSetSeed) {
        const int skip = __builtin_amdgcn_readlane(rec.x, 0);
        if (w == 0) {
          double2 p = make_double2(1.0, 0.0);
          for (int j = 0; j < net.n_comp; ++j)
            if (j != skip) p = cmul(p, scal[j]);
          m[hdr >> 16] = from_d2<V>(p);
        }
      } else if (GRAD && type == kSetLeafGrad) {
        set_leafgrad<V>(m, dv, gacc, rec, hdr, w);
      }
      __syncthreads();
      rec = rec1;
      rec1 = nrec;
    }

    if (valid && w == 0) {
      double2 p = make_double2(1.0, 0.0);
      for (int j = 0; j < net.n_comp; ++j) p = cmul(p, scal[j]);
      double *ov = a.out_val + ((size_t)ni * a.n_sets + set) * 2;
      ov[0] = p.x;
      ov[1] = p.y;
    }
    if (GRAD && valid)
      for (int p = w; p < a.n_params; p += W)
        a.out_grad[((size_t)ni * a.n_sets + set) * a.n_params + p] = gacc[p];
    __syncthreads();
  }
}

// obj[s] = offset + sum_i coef[i] Re(val[i][s]); grad[s][p] = sum_i coef[i] gnet[i][s][p].
// One 64-lane wave per (set, quantity): lane partial sums in network order,
// then the fixed DPP tree; FP64 throughout.
__global__ __launch_bounds__(64) void combine_kernel(const double *__restrict__ val, const double *__restrict__ gnet,
                                                     const double *__restrict__ coef, double offset, int n_nets,
                                                     int n_sets, int n_params, double *obj, double *grad) {
  const int nq = n_params + 1;
  const int s = blockIdx.x / nq, q = (int)(blockIdx.x % nq) - 1;
  if ((q < 0 && !obj) || (q >= 0 && !grad)) return;  // uniform over the wave
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_nets; i += 64)
    acc += coef[i] * (q < 0 ? val[((size_t)i * n_sets + s) * 2] : gnet[((size_t)i * n_sets + s) * n_params + q]);
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    if (q < 0) obj[s] = offset + acc;
    else grad[(size_t)s * n_params + q] = acc;
  }
}

// --- launch helpers (host) ----------------------------------------------------------------
template <typename T, bool G>
static const void *fused_ptr_t(int block, bool rec_only, bool gmem) {
  if (gmem) return (const void *)fused_exec_kernel<T, 256, G, false, true>;
  switch (block) {
    case 64:
      return rec_only ? (const void *)fused_exec_kernel<T, 64, G, true, false>
                      : (const void *)fused_exec_kernel<T, 64, G, false, false>;
    case 128: return (const void *)fused_exec_kernel<T, 128, G, false, false>;
    default: return (const void *)fused_exec_kernel<T, 256, G, false, false>;
  }
}

// gmem: the global-arena instance (256 lanes)
const void *fused_kernel_ptr(int dtype, int block, bool grad, bool rec_only, bool gmem) {
  if (dtype == TN_C128)
    return grad ? fused_ptr_t<double, true>(block, rec_only, gmem) : fused_ptr_t<double, false>(block, rec_only, gmem);
  return grad ? fused_ptr_t<float, true>(block, rec_only, gmem) : fused_ptr_t<float, false>(block, rec_only, gmem);
}

hipError_t launch_fused(int dtype, int block, bool grad, bool rec_only, bool gmem, const FusedArgs &a, int grid,
                        int lds_bytes, hipStream_t st) {
  const void *k = fused_kernel_ptr(dtype, block, grad, rec_only, gmem);
  void *args[] = {(void *)&a};
  return hipLaunchKernel(k, dim3(grid), dim3(gmem ? 256 : block), args, lds_bytes, st);
}

template <typename T, bool G>
static const void *fused_sets_ptr_t(int sets) {
  return sets == 2 ? (const void *)fused_sets_kernel<T, G, 5> : (const void *)fused_sets_kernel<T, G, 4>;
}

// sets: angle sets per wave (2 or 4)
const void *fused_sets_kernel_ptr(int dtype, bool grad, int sets) {
  if (dtype == TN_C128) return grad ? fused_sets_ptr_t<double, true>(sets) : fused_sets_ptr_t<double, false>(sets);
  return grad ? fused_sets_ptr_t<float, true>(sets) : fused_sets_ptr_t<float, false>(sets);
}

hipError_t launch_fused_sets(int dtype, bool grad, int sets, const FusedArgs &a, int grid, int lds_bytes, hipStream_t st) {
  const void *k = fused_sets_kernel_ptr(dtype, grad, sets);
  void *args[] = {(void *)&a};
  return hipLaunchKernel(k, dim3(grid), dim3(64), args, lds_bytes, st);
}

hipError_t launch_combine(const double *val, const double *gnet, const double *coef, double offset, int n_nets,
                          int n_sets, int n_params, double *obj, double *grad, hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(n_sets * (n_params + 1)), dim3(64), 0, st, val, gnet, coef, offset, n_nets,
                     n_sets, n_params, obj, grad);
  return hipGetLastError();
}

hipError_t launch_bind(int dtype, const DParam *slots, int n_slots, const double *params, int n_params, int n_sets,
                       int per_set, void *G, void *dG, hipStream_t st) {
  if (n_slots == 0) return hipSuccess;
  dim3 grid(n_slots, n_sets);
  if (dtype == TN_C128)
    hipLaunchKernelGGL(bind_params_kernel<double2>, grid, dim3(256), 0, st, slots, params, n_params, per_set,
                       (double2 *)G, (double2 *)dG);
  else
    hipLaunchKernelGGL(bind_params_kernel<float2>, grid, dim3(256), 0, st, slots, params, n_params, per_set,
                       (float2 *)G, (float2 *)dG);
  return hipGetLastError();
}

}  // namespace qtn
