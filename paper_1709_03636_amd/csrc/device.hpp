// Device-side program format shared by the runtime and the kernels.
#pragma once
#include <cstdint>

#include "../../include/qtn.h"

namespace qtn {

// One op of a compiled network program, as the kernels read it (56 bytes).
// Offsets are in complex elements of the executor's memory (LDS for the
// fused executor, a per-set global arena for the level executor). Output
// index c = (i, b, j): i the nFX X-only bits (deposited at maskX in X), b
// the nB batch bits (offsets from the table at tabB), j the nFY Y-only bits
// (deposited at maskY in Y).
struct DOp {
  int32_t type;      // OpType
  int64_t x, y, z;   // operand / result offsets (OP_SCALAR: z = scalar slot); 64-bit: a level
                     // network's region may pass 2^31 elements (2^30-entry intermediates)
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
  int32_t off, slot, diag, pad;  // diag: only the diagonal of the gate (2^bits entries)
  int64_t goff;                  // 64-bit: a level network's adjoint accumulators may sit past 2^31
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
//               of lanes 1-2 the FP64 coefficient;
//  kRecAcc      (task executor) adjoint of a parametric leaf, 2^B <= 256
//               entries, added into its accumulator at the header's
//               offset: x = offset of entry l, y = canonical indices of
//               entries l + 64 q (8 bits each).
// Type 0: the op runs from its DOp descriptor.
constexpr int kRecLite = 1, kRecWide = 2, kRecNarrow = 3, kRecScalar = 4, kRecSeed = 5, kRecLeafGrad = 6, kRecAcc = 7;
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

// Level executor: every op of a network program too large for LDS is an
// item of workgroup-sized tasks (rank 0..count-1) working in the network's
// region of the level arena (`base` elements from its start, `stride`
// elements per parameter vector). Item mode launches the items of a network
// one by one, each over all parameter vectors on the whole chip; the task
// executor runs whole (network, parameter vector) programs, one per
// workgroup, with items built for one vector (TNet).
enum PKind : int32_t {
  PK_SETUP = 0,       // constants and bound parametric tensors into the region, adjoint accumulators cleared
  PK_THIN = 1,        // thin contraction (eq. (1)) or leaf adjoint on the vector units
  PK_MFMA = 2,        // contraction as a complex GEMM on the matrix cores
  PK_SPLITSUM = 3,    // sum of the partial tiles of a split matrix-core product, in range order (FP64)
  PK_SCALAR = 4,      // rank-0 result: partial sums of the summed index (FP64)
  PK_SCALAR_SUM = 5,  // rank-0 result: sum of the partial sums in index order (FP64)
  PK_SEED = 6,        // adjoint seed: product of the other component scalars
  PK_FINISH = 7,      // value and gradient of the network into the outputs
  PK_TREC = 8         // task executor: lgl steps of small thin contractions or leaf adjoint
                      // additions from lane records rec, rec + 1, ..., operands in the
                      // workgroup's LDS arena; step t runs 1-4 independent records (wave w the
                      // w-th), its count less one in bits 2(t mod 16) of a(t / 16); count: the
                      // first step's
};

struct PItem {
  DOp op;
  DRuns ru;
  int64_t base;    // the network's arena region (elements)
  int64_t stride;  // elements per parameter vector
  int64_t zs;      // MFMA (split) and SPLITSUM: partial tiles from this element of the split scratch;
                   // SCALAR / SCALAR_SUM: partial sums from this double of the partial-sum buffer
  int64_t sbase;   // the network's component scalars (doubles; [set][n_comp] complex)
  int32_t kind;    // PKind
  int32_t count;   // tasks of the item (workgroups of a one-item launch)
  int32_t lgl;     // THIN: 2^lgl lanes per output (< 0: four outputs per lane); MFMA / SPLITSUM: log2 of the
                   // summed-index ranges; SCALAR: workgroups per parameter vector (1: writes the scalar)
  int32_t mv;      // MFMA: kernel variant (tile shape, operand layouts)
  int32_t n_comp;  // component scalars of the network
  int32_t a0, a1, a2, a3, a4, a5;  // SETUP: const_begin, n_const, ptens_begin, n_pt, -, zero_n (zero_begin: zs);
                                   // FINISH: network index, ptens_begin, n_pt; THIN: see kLdsX
  int32_t rec;     // task executor: this item's first lane record (PK_TREC), else -1
  int32_t nrec;    // task executor: the next item's first lane record (loaded while this item runs), else -1
  int32_t nrec_n;  // and how many it has (PK_TREC: up to 4 independent contractions, one per wave)
};

// Task executor: a workgroup keeps the small tensors of its program in an
// LDS arena of kLdsArenaBytes. SETUP with mv = 1 also copies the leaf
// region (constants and bound parametric tensors) to LDS [0, leaf region).
// A THIN item's a0 says which operands live there: kLdsX / kLdsY / kLdsZ
// (op.x / op.y / op.z are then LDS element offsets; a leaf adjoint's
// accumulator is its Y); kPackedTab: the summed-index offsets come from the
// bit positions in a1 (X) and a2 (Y), 5 bits per summed bit, lowest first,
// instead of the table (nS <= 6). With gradients the adjoint accumulators
// may live in LDS too, as one block at LDS element a4 of SETUP (mv bit 1),
// which clears it there instead of in the region; FINISH (mv = 1) then reads
// the accumulator of region offset goff at LDS a3 + goff - zs.
constexpr int kLdsX = 1, kLdsY = 2, kLdsZ = 4, kPackedTab = 8;
// A MFMA item's mv bit kMfmaPacked (bits 0-3: tile variant, 4-5:
// precision): every summed bit's X and Y offset is a power of two, and a0 ..
// a5 hold their bit positions (5 bits each, six per word; X in a0 .. a2, Y
// in a3 .. a5), read instead of the offset table; nS <= 18.
constexpr int kMfmaPacked = 64;
constexpr int kMaxRunSteps = 96;  // steps of one PK_TREC item (2 bits each in a0 .. a5)
// LDS of a matrix-core tile (the largest, 64 x 64, with 16 summed entries
// per stage): split-BF16 four 64-row planes of 20 dwords; FP32 / FP64 the
// X tile (64 rows of 17 entries) and the Y tile (16 rows of 66). The task
// executor lays it after its arena; between the items that use it (matrix
// cores; rank-0 sums and outputs use its first kTileReserve bytes) the
// planner may place tensors there, from element kLdsArenaBytes / e +
// kTileReserve / e.
template <int PREC>
constexpr int kTileLdsBytes = PREC == TN_MFMA_BF16X3 ? 4 * 64 * 20 * 4 : (64 * 17 + 16 * 66) * (PREC == TN_MFMA_FP64 ? 16 : 8);
constexpr int kTileReserve = 1024;
constexpr int kPackedTabBits = 6;
template <int PREC>
constexpr int kLdsArenaBytes = PREC == TN_MFMA_FP64 ? 24576 : 32768;  // complex128: its tiles take more LDS

// One network of a task-executor launch: task (network j, vector s) runs
// items [item0, item0 + n_items) (built for one vector) on the vector's
// slice of the network's region.
struct TNet {
  int64_t abase;   // arena region (elements): vector s at abase + s * stride
  int64_t stride;  // elements per parameter vector
  int64_t sbase;   // component scalars (doubles): vector s at sbase + s * n_comp * 2
  int32_t item0, n_items, n_comp, pad;
};

// Workgroups per parameter vector of a large rank-0 contraction.
constexpr int kScalarParts = 256;

}  // namespace qtn
