// Internal data structures of the contraction library (host side).
//
// A circuit becomes a closed network of leaf tensors joined by wires
// (Sec. Preliminaries of the paper). Internally every wire is split into
// bit labels: a dimension-4 wire of the folded network carries two bits
// (ket bit = high bit, bra bit = low bit, so wire value 2a+b is rho_ab) and a
// dimension-2 wire of the amplitude network carries one bit. Tensors are
// stored densely, row-major over their label list (first label = most
// significant address bit), as interleaved complex numbers.
//
// A contraction order is compiled into a linear program of ops over buffers
// (leaves, intermediates, adjoints, scalars); both executors (the fused
// per-workgroup one and the level-synchronous one) run the same program.
#pragma once
#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qtn.h"

namespace qtn {

using cd = std::complex<double>;

// Summed-index offset tables are split in a low part of at most this many
// bits and a high part (see Op::tab).
constexpr int kTabLoBits = 12;
// Largest intermediate (log2 entries) a plan may create: 32-bit addressing.
constexpr int kMaxTensorBits = 31;

// Op types of the compiled program.
enum OpType : int32_t {
  OP_CONTRACT = 0,  // Z[F_X, F_Y] = sum_S X[F_X, S] Y[S, F_Y]   (eq. (1))
  OP_SCALAR = 1,    // rank-0 result, accumulated in FP64 into a scalar slot
  OP_SEED = 2,      // adjoint seed of component `aux0`: product of the other scalars
  OP_LEAFGRAD = 3   // grad[param] += coeff * Re sum Gbar . dG/dtheta
};

// A parametric tensor: the (super)operator of exp(-i theta P / 2) with
// theta = coeff * params[param]. Pauli P = X, Y, Z (one qubit) or Z(x)Z.
struct ParamTensor {
  int kind;      // TN_RX, TN_RY, TN_RZ, TN_ZZ
  int param;
  double coeff;
  int folded;    // 1: superoperator U (x) conj(U); 0: the matrix U
  int bits;      // log2(entries)
  int diag = 0;  // 1: only the diagonal (a gate diagonal in the computational basis on hyperedge wires)
};

struct Leaf {
  std::vector<int> wires;  // storage order, first = most significant
  int src;                 // >= 0: constant id; < 0: -(param tensor id) - 1
};

// One op of the compiled program. Buffers are numbered: leaves first
// (0..n_leaves-1), then intermediates and adjoints in creation order.
struct Op {
  OpType type;
  int x, y, z;            // buffer ids (z: scalar slot for OP_SCALAR; component for OP_SEED)
  int nFX, nS, nFY;       // bits: free of X only, summed, free of Y only
  int nB = 0;             // batch bits: shared by X and Y and kept in Z (hyperedges)
  uint32_t maskX_F = 0, maskY_F = 0;  // address positions of the X-only / Y-only free bits
  std::vector<int32_t> tabB;  // (X, Y) offset pairs of the batch index b (2^nB pairs; empty if nB = 0)
  std::vector<int32_t> tab;  // OP_CONTRACT/OP_SCALAR: (X, Y) offset pairs of the summed index k:
                             //   2^min(nS,12) pairs for the low bits of k, then (nS > 12)
                             //   2^(nS-12) pairs for the high bits; offsets add
                             // OP_LEAFGRAD: 2^bits canonical index per buffer index
  int aux0 = 0, aux1 = 0; // OP_LEAFGRAD: param tensor id, leaf id; OP_SEED: component
  bool fwd = true;        // part of the forward pass
};

struct Plan {
  std::vector<Op> ops;                       // forward ops then (grad) reverse ops
  int n_fwd_ops = 0;
  std::vector<std::vector<int>> labels;      // per buffer
  std::vector<int> buf_bits;                 // log2 entries per buffer
  int n_leaves = 0;
  int n_components = 0;
  std::vector<int> comp_root_step;           // op index producing each component scalar
  std::vector<int> seed_buf;                 // grad: rank-0 adjoint buffer per component
  int n_steps = 0;                           // forward pairwise contractions
  int peak_bits = 0, max_rank_wires = 0;
  double flops = 0, bytes = 0;               // forward, one angle set
  double flops_grad = 0, bytes_grad = 0;     // reverse ops only
  double peak_live_bytes = 0;
  int recompute_runs = 1;                    // grad: forward runs recomputed before their adjoints (1: none)
  std::vector<std::array<int, 3>> step_dims; // forward (nFX, nS, nFY)
};

struct Net {
  int n_qubits = 0, mode = 0, dtype = 0, n_params = 0, wire_bits = 2;
  std::vector<Leaf> leaves;
  std::vector<std::vector<int>> wire_holders; // leaf ids holding each wire (2, or more for a hyperedge)
  std::vector<std::vector<cd>> consts;        // distinct constant tensors
  std::vector<ParamTensor> ptensors;          // distinct parametric tensors
  uint64_t mem_limit = 64ull << 30;
  bool has_order = false;
  std::vector<int> order;
  Plan plan;       // forward only
  Plan gplan;      // forward + reverse (adjoint)
  void *dev = nullptr;  // device-side cache (runtime)
  bool poisoned = false;
  int elem_bytes() const { return dtype == TN_C128 ? 16 : 8; }
};

// --- shared helpers ---------------------------------------------------------
void set_error(const std::string &msg);

// State-vector comparator (sv.hip).
int64_t sv_workspace_bytes(int n);
int sv_maxcut_p1(int n, const int32_t *edges, int n_edges, double gamma, double beta, void *workspace,
                 int64_t ws_bytes, double *cost, void *stream);

struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint32_t below(uint32_t m) { return (uint32_t)(((next() >> 32) * (uint64_t)m) >> 32); }
};

// build.cpp
int build_network(const tn_gate *gates, int n_gates, int n_qubits, const double *init,
                  const tn_target *target, int n_params, int dtype, Net &net);

// order.cpp
int order_stochastic(const Net &net, uint64_t seed, int max_rej, std::vector<int> &pi);
int order_linegraph(const Net &net, int trials, double budget_s, uint64_t seed, std::vector<int> &pi);

// plan.cpp
struct OrderCost {
  int peak_bits = 0, max_rank_wires = 0;
  double flops = 0;
};
OrderCost order_cost(const Net &net, const std::vector<int> &pi);

// First-fit arena allocator over element offsets.
struct Arena {
  std::vector<std::pair<int64_t, int64_t>> free_;  // (offset, size), sorted by offset
  int64_t top = 0;
  int64_t alloc(int64_t n);
  void release(int64_t off, int64_t n);
};

// Offsets of the buffers >= n_leaves written by ops [0, n_ops) of a plan,
// reusing memory by liveness; returns the elements needed.
int64_t layout_buffers(const Plan &p, int n_ops, std::vector<int64_t> &off);

int compile_plan(const Net &net, const std::vector<int> &pi, bool with_grad, Plan &plan);

}  // namespace qtn
