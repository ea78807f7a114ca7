// Device-side program format shared by the runtime and the kernels.
#pragma once
#include <cstdint>

namespace qtn {

// One op of a compiled network program, as the kernels read it (56 bytes).
// Offsets are in complex elements of the executor's memory (LDS for the
// fused executor, a per-set global arena for the level executor). Output
// index c = (i, b, j): i the nFX X-only bits (deposited at maskX in X), b
// the nB batch bits (offsets from the table at tabB), j the nFY Y-only bits
// (deposited at maskY in Y).
struct DOp {
  int32_t type;      // OpType
  int32_t x, y, z;   // operand / result offsets (OP_SCALAR: z = scalar slot)
  int32_t nFX, nS, nFY;
  uint32_t maskX, maskY;
  int32_t tab;       // offset into the int32 table array (summed index)
  int32_t aux0, aux1;
  int32_t nB, tabB;  // batch bits and their (X, Y) offset table
};

// The free-bit masks of an op as runs of consecutive address bits, lowest
// first, packed (shift | len << 8 | pos << 16): deposit(v) = OR over runs of
// bits [shift, shift+len) of v moved to [pos, pos+len). Unused runs have
// len 0; runsX[0] == -1 when the mask has more than kMaxRuns runs. Passed to
// the level executor's kernels with each launch.
struct DRuns {
  int32_t runsX[4], runsY[4];
};
constexpr int kMaxRuns = 4;

// Runs of a bit mask in the DOp encoding (host and device).
inline void pack_runs(uint32_t mask, int32_t out[4]) {
  int n = 0, shift = 0;
  for (int j = 0; j < 4; ++j) out[j] = 0;
  int p = 0;
  while (p < 32) {
    if (!((mask >> p) & 1u)) { ++p; continue; }
    int q = p;
    while (q < 32 && ((mask >> q) & 1u)) ++q;
    if (n == 4) { out[0] = -1; return; }
    out[n++] = shift | ((q - p) << 8) | (p << 16);
    shift += q - p;
    p = q;
  }
}

// A parametric tensor: entries of exp(-i theta P / 2) (folded: its
// superoperator) with theta = coeff * params[param]. In the binding kernel
// `off` is its offset in a parameter vector's slice of the bound-tensor
// buffer; in a network program `off` is its place in executor memory,
// `goff` that of its adjoint accumulator and `slot` its offset in the
// bound-tensor slice.
struct DParam {
  int32_t kind, param, folded, bits;
  int32_t off, goff, slot, diag;  // diag: only the diagonal of the gate (2^bits entries)
  double coeff;
};

// One network program (forward, or forward + adjoint).
struct DNet {
  int32_t op_begin, n_ops;      // into the op array
  int32_t rec_begin;            // lane records of op o at (rec_begin + o) * 64
  int32_t n_comp;               // component scalars
  int32_t mem_elems;            // executor memory (elements) incl. leaves
  int32_t const_begin, n_const; // constant leaf values: global -> [0, n_const)
  int32_t ptens_begin, n_ptens; // DParam range
};


// Lane record of an op of the fused executor (64 lanes per op, one int4
// each, lane l holding (x, y, z, w)). w of lane 0 is a workgroup-uniform
// header: bits 0-2 the record type, three 4-bit fields A (bits 3-6), B
// (7-10), C (11-14), and bits 15.. the result offset (leaf gradients: the
// parameter index). Offsets are LDS element offsets; "packed" means an
// (X, Y) pair as two 16-bit halves. Types:
//  kRecLite     contraction, 2^B <= 64 outputs, K = 2^A <= 4 summed
//               entries (larger K go to kRecNarrow, which needs fewer
//               registers): x, y = offsets of output l's X and Y rows, z =
//               packed offsets of summed entry l;
//  kRecWide     outer product (K = 1), 2^B <= 256 outputs: x, y for output
//               l; w of lanes 1-3 = packed offset steps of outputs 64 l
//               (offsets add over disjoint index bits);
//  kRecNarrow   contraction, 2^B <= 64 outputs, K = G R with G = 2^A lanes
//               per output and R = 2^C entries per lane: lane l serves
//               output l / G, its x, y include the offsets of entry l mod G,
//               z of lane i = packed offsets of entry G i; the G partial
//               sums are reduced across lanes;
//  kRecScalar   rank-0 result, K = 2^A <= 64: x, y = offsets of entry l;
//               FP64 products and sum;
//  kRecSeed     adjoint seed: x of lane 0 = the component left out;
//  kRecLeafGrad adjoint of a parametric leaf, 2^B <= 256 entries: x =
//               offset of entry l, y = canonical indices of entries
//               l + 64 q (8 bits each), z of lane 0 the bound-tensor slot,
//               of lanes 1-2 the FP64 coefficient.
// Type 0: the op runs from its DOp descriptor.
constexpr int kRecLite = 1, kRecWide = 2, kRecNarrow = 3, kRecScalar = 4, kRecSeed = 5, kRecLeafGrad = 6;
constexpr int kRecLanes = 64;

// Set-packed records: one 64-lane wave runs S = 2 or 4 angle sets of one
// network at once, W = 64 / S lanes per set, each set in its own LDS region
// of set_stride elements. A record is W int4 (lane w: x, y, z, w); lane w of
// every set reads lane w of the record. Header (w of lane 0): bits 0-2
// type, 3-5 log2 G, 6-8 log2 Q, 9-11 log2 R, 12-15 log2 of the number of
// outputs, 16.. the result offset (leaf gradient: parameter index).
// "Packed" = two 16-bit offsets (X, Y). G <= kMaxGroupLanes keeps every
// cross-lane sum inside one row of 16 lanes.
//  kSetContract  lane w serves outputs w / G + (W / G) q (q < Q) and summed
//                entries w mod G + G i (i < R): x, y = operand offsets of
//                its first output and entry; z of lane i = packed offset
//                step of entry G i; w of lane q >= 1 = packed offset step of
//                output W q (Q > 1 only when G = 1). The G partial sums of
//                an output are reduced across lanes.
//  kSetScalar    rank-0 result in FP64 over entries w + G i; x, y, z as
//                above.
//  kSetSeed      adjoint seed; x of lane 0 = the component left out.
//  kSetLeafGrad  adjoint of a parametric leaf against the bound angle
//                derivative, FP64, entries w + G i: x = adjoint offset of
//                entry w, y = derivative index of entry w, z of lane i =
//                index step of entry G i, w of lane 1 = bound-tensor slot,
//                of lanes 2-3 = FP64 coefficient.
// Offsets add over disjoint index bits, which the host checks per op.
constexpr int kMaxGroupLanes = 16, kLgMaxGroupLanes = 4;
constexpr int kSetContract = 1, kSetScalar = 2, kSetSeed = 3, kSetLeafGrad = 4;

// One step of one network for the grouped level launches: every network
// works in its own region of the level arena (`base` elements from its
// start, `stride` elements per parameter vector).
// Workgroups [blk0, next item's blk0) of a grouped launch serve the item;
// a thin contraction sums each output on 2^lgl lanes (lgl < 0: a lane
// computes four consecutive outputs); a matrix-core product splits its
// summed index into 2^lgl ranges, whose partial results go to a scratch
// buffer from element zs.
struct LItem {
  DOp op;
  DRuns ru;
  int64_t base, stride, zs;
  int32_t blk0, lgl;
};

// Arguments of the fused executor kernel.
struct FusedArgs {
  const DNet *nets;
  const DOp *ops;
  const int4 *recs;
  const int32_t *tabs;
  const void *consts;
  const DParam *ptens;
  const void *bound;        // [set][per_set] parametric tensors (binding kernel output)
  const void *dbound;       // [set][per_set] their angle derivatives (adjoint programs)
  const int32_t *task_net;  // queue position -> network index (cost order)
  double *out_val;          // [net][set][2]
  double *out_grad;         // [net][set][n_params] (adjoint programs)
  int n_params, n_sets, n_tasks, per_set;
  int set_stride, n_groups, max_comp;  // set-packed executor: LDS elements per set, set groups, scalars per set
  int per_block;            // workgroup b runs tasks [b*per_block, (b+1)*per_block)
  void *garena;             // global-arena executor: workgroup b works in garena + b * garena_stride
  int64_t garena_stride;    // (elements)
  int scratch_off, scal_off, gacc_off, red_off, gbar_off;  // LDS byte offsets
};

// Arguments of the level executor kernels (one chunk of parameter vectors).
struct LevelArgs {
  void *arena;     // [set][stride] elements
  int64_t stride;  // elements per parameter vector
  int n_sets;      // parameter vectors in this chunk
  double *scal;    // [set][n_comp] component scalars (complex, FP64)
  int n_comp;
  double *part;    // [set][kScalarParts] partial sums of a large rank-0 contraction
};

// Workgroups per parameter vector for a large rank-0 contraction.
constexpr int kScalarParts = 256;

}  // namespace qtn
