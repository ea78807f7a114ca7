// Circuit -> closed tensor network (Sec. Preliminaries of the paper).
//
// Nodes: one initial-state tensor per qubit, one tensor per gate and one
// measurement tensor per qubit; the network's connectivity is the circuit's.
// Folded form (PROBABILITY / EXPECTATION): wires of dimension 4 carry the
// vectorised density matrix [rho00, rho01, rho10, rho11]; a gate U acting as
// rho -> U rho U^dagger is the superoperator with entries U_ac conj(U_bd)
// from input (c, d) to output (a, b); the measurement of an operator P is the
// vector whose entry 2a+b is P_ba, so its contraction gives Tr(P rho).
// Unfolded form (AMPLITUDE): dimension-2 wires, gate matrices, <x| outputs.
#include <cmath>
#include <cstring>
#include <map>
#include <set>

#include "internal.hpp"

namespace qtn {

namespace {

using Mat = std::vector<cd>;  // row-major, dim x dim

const cd I1(0.0, 1.0);

Mat pauli(int which) {  // 0 = I, 1 = X, 2 = Y, 3 = Z
  switch (which) {
    case 1: return {0, 1, 1, 0};
    case 2: return {0, -I1, I1, 0};
    case 3: return {1, 0, 0, -1};
    default: return {1, 0, 0, 1};
  }
}

Mat kron(const Mat &a, const Mat &b, int da, int db) {
  Mat r((size_t)da * db * da * db);
  for (int i = 0; i < da; ++i)
    for (int j = 0; j < da; ++j)
      for (int k = 0; k < db; ++k)
        for (int l = 0; l < db; ++l) r[(size_t)(i * db + k) * (da * db) + (j * db + l)] = a[i * da + j] * b[k * db + l];
  return r;
}

// exp(-i theta P / 2) for a Pauli (product) P with P^2 = I.
Mat rotation(const Mat &P, int dim, double theta) {
  Mat r(P.size());
  double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) r[i * dim + j] = (i == j ? cd(c, 0) : cd(0, 0)) - I1 * s * P[i * dim + j];
  return r;
}

const Mat &pauli_of_kind(int kind, int &dim) {
  static const Mat X = pauli(1), Y = pauli(2), Z = pauli(3), ZZ = kron(pauli(3), pauli(3), 2, 2);
  dim = 2;
  switch (kind) {
    case TN_RX: return X;
    case TN_RY: return Y;
    case TN_RZ: return Z;
    default: dim = 4; return ZZ;
  }
}

bool gate_is_2q(int kind) { return kind == TN_ZZ || kind == TN_CNOT || kind == TN_CZ || kind == TN_U2 || kind == TN_SUPER2; }
bool gate_is_super(int kind) { return kind == TN_SUPER1 || kind == TN_SUPER2; }
bool gate_is_param(int kind) { return kind == TN_RX || kind == TN_RY || kind == TN_RZ || kind == TN_ZZ; }

// Fixed matrix of a gate (parametric kinds evaluated at theta).
Mat gate_matrix(const tn_gate &g, double theta) {
  const double h = 1.0 / std::sqrt(2.0);
  switch (g.kind) {
    case TN_H: return {h, h, h, -h};
    case TN_X: return pauli(1);
    case TN_Y: return pauli(2);
    case TN_Z: return pauli(3);
    case TN_CNOT: return {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0};
    case TN_CZ: return {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, -1};
    case TN_U1:
    case TN_U2:
    case TN_SUPER1:
    case TN_SUPER2: {
      int dim = g.kind == TN_U1 ? 2 : (g.kind == TN_U2 ? 4 : (g.kind == TN_SUPER1 ? 4 : 16));
      Mat m((size_t)dim * dim);
      for (int i = 0; i < dim * dim; ++i) m[i] = cd(g.matrix[2 * i], g.matrix[2 * i + 1]);
      return m;
    }
    default: {
      int dim;
      const Mat &P = pauli_of_kind(g.kind, dim);
      return rotation(P, dim, theta);
    }
  }
}

bool is_diag_matrix(const Mat &m, int dim) {
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j)
      if (i != j && std::abs(m[i * dim + j]) != 0.0) return false;
  return true;
}

// Diagonal in the computational basis (such gates commute with each other).
bool gate_is_diagonal(const tn_gate &g) {
  switch (g.kind) {
    case TN_Z: case TN_RZ: case TN_ZZ: case TN_CZ: return true;
    case TN_U1: return is_diag_matrix(gate_matrix(g, 0.0), 2);
    case TN_U2: return is_diag_matrix(gate_matrix(g, 0.0), 4);
    default: return false;
  }
}

bool is_unitary(const Mat &m, int dim) {
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) {
      cd s = 0;
      for (int k = 0; k < dim; ++k) s += m[i * dim + k] * std::conj(m[j * dim + k]);
      if (std::abs(s - (i == j ? 1.0 : 0.0)) > 1e-10) return false;
    }
  return true;
}

// A folded superoperator preserves the trace: summing its output over the
// diagonal (a = b on every qubit) leaves the trace functional of the input.
bool is_trace_preserving(const Mat &S, int qubits) {
  const int nin = qubits == 1 ? 4 : 16;
  for (int in = 0; in < nin; ++in) {
    cd s = 0;
    if (qubits == 1) {
      for (int a = 0; a < 2; ++a) s += S[(3 * a) * 4 + in];
    } else {
      for (int a0 = 0; a0 < 2; ++a0)
        for (int a1 = 0; a1 < 2; ++a1) s += S[((3 * a0) * 4 + 3 * a1) * 16 + in];
    }
    const bool diag = qubits == 1 ? (in == 0 || in == 3) : ((in >> 2) == 0 || (in >> 2) == 3) && ((in & 3) == 0 || (in & 3) == 3);
    if (std::abs(s - (diag ? 1.0 : 0.0)) > 1e-10) return false;
  }
  return true;
}

// Superoperator of a one-qubit gate, wires (out, in): entry index
// (2a+b)*4 + (2c+d) holds U_ac conj(U_bd).
Mat superop_1q(const Mat &U) {
  Mat S(16);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) S[(2 * a + b) * 4 + (2 * c + d)] = U[a * 2 + c] * std::conj(U[b * 2 + d]);
  return S;
}

// Superoperator of a two-qubit gate, wires (q0 out, q1 out, q0 in, q1 in):
// entry ((2a0+b0)*4 + (2a1+b1))*16 + (2c0+d0)*4 + (2c1+d1) holds
// U[(a0 a1),(c0 c1)] conj(U[(b0 b1),(d0 d1)]).
Mat superop_2q(const Mat &U) {
  Mat S(256);
  for (int idx = 0; idx < 256; ++idx) {
    int a0 = (idx >> 7) & 1, b0 = (idx >> 6) & 1, a1 = (idx >> 5) & 1, b1 = (idx >> 4) & 1;
    int c0 = (idx >> 3) & 1, d0 = (idx >> 2) & 1, c1 = (idx >> 1) & 1, d1 = idx & 1;
    S[idx] = U[(2 * a0 + a1) * 4 + (2 * c0 + c1)] * std::conj(U[(2 * b0 + b1) * 4 + (2 * d0 + d1)]);
  }
  return S;
}

// Diagonal of a gate that is diagonal in the computational basis, as a
// tensor over its (input = output) wires: folded, entry 2a+b (one qubit) or
// (2a0+b0)*4 + (2a1+b1) (two) holds U_aa conj(U_bb); unfolded, entry a
// (or 2a0+a1) holds U_aa.
Mat diag_entries(const Mat &U, bool two, bool folded) {
  const int dim = two ? 4 : 2;
  Mat d;
  if (!folded) {
    for (int a = 0; a < dim; ++a) d.push_back(U[a * dim + a]);
    return d;
  }
  if (!two) {
    for (int a = 0; a < 2; ++a)
      for (int bb = 0; bb < 2; ++bb) d.push_back(U[a * 2 + a] * std::conj(U[bb * 2 + bb]));
    return d;
  }
  d.resize(16);
  for (int e = 0; e < 16; ++e) {
    const int a0 = (e >> 3) & 1, b0 = (e >> 2) & 1, a1 = (e >> 1) & 1, b1 = e & 1;
    const int ka = 2 * a0 + a1, kb = 2 * b0 + b1;
    d[e] = U[ka * 4 + ka] * std::conj(U[kb * 4 + kb]);
  }
  return d;
}

struct Builder {
  Net &net;
  std::map<std::vector<double>, int> const_ids;
  std::map<std::tuple<int, int, double, int>, int> ptensor_ids;
  explicit Builder(Net &n) : net(n) {}

  int new_wire() {
    net.wire_holders.emplace_back();
    return (int)net.wire_holders.size() - 1;
  }
  int add_const(const Mat &m) {
    std::vector<double> key;
    key.reserve(2 * m.size());
    for (auto &x : m) {
      key.push_back(x.real() == 0.0 ? 0.0 : x.real());  // fold -0.0 into 0.0
      key.push_back(x.imag() == 0.0 ? 0.0 : x.imag());
    }
    auto it = const_ids.find(key);
    if (it != const_ids.end()) return it->second;
    net.consts.push_back(m);
    int id = (int)net.consts.size() - 1;
    const_ids[key] = id;
    return id;
  }
  int add_ptensor(int kind, int param, double coeff, int folded, int diag) {
    auto key = std::make_tuple(kind, param, coeff, folded + 2 * diag);
    auto it = ptensor_ids.find(key);
    if (it != ptensor_ids.end()) return it->second;
    int nq = kind == TN_ZZ ? 2 : 1;
    int bits = (folded ? 2 : 1) * (diag ? 1 : 2) * nq;
    net.ptensors.push_back({kind, param, coeff, folded, bits, diag});
    int id = (int)net.ptensors.size() - 1;
    ptensor_ids[key] = id;
    return id;
  }
  void add_leaf(const std::vector<int> &wires, int src) {
    int id = (int)net.leaves.size();
    net.leaves.push_back({wires, src});
    for (int w : wires) net.wire_holders[w].push_back(id);
  }
};

}  // namespace

// Folded superoperator of a channel given by Kraus operators E_k (d x d,
// d = 2 or 4, row-major interleaved re/im): one qubit, entry
// [(2a+b)*4 + (2c+d)] = sum_k E_k[a][c] conj(E_k[b][d]); two qubits, with
// each of a, b, c, d split into (qubit q0 bit, qubit q1 bit), entry
// [((2a0+b0)*4 + (2a1+b1))*16 + (2c0+d0)*4 + (2c1+d1)] =
// sum_k E_k[2a0+a1][2c0+c1] conj(E_k[2b0+b1][2d0+d1]).
static std::vector<double> fold_kraus(const double *m, int n_k, bool two) {
  const int dim = two ? 4 : 2, q = two ? 2 : 1, sdim = 1 << (2 * q);
  std::vector<cd> S((size_t)sdim * sdim, cd(0.0, 0.0));
  for (int k = 0; k < n_k; ++k) {
    const double *e = m + (size_t)k * 2 * dim * dim;
    auto E = [&](int r, int c) { return cd(e[2 * (r * dim + c)], e[2 * (r * dim + c) + 1]); };
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b)
        for (int c = 0; c < dim; ++c)
          for (int d = 0; d < dim; ++d) {
            // folded wire value of qubit j: 2 * (ket bit) + (bra bit)
            int row = 0, col = 0;
            for (int j = 0; j < q; ++j) {
              const int sh = q - 1 - j;  // qubit q0 is the most significant bit
              row = row * 4 + 2 * ((a >> sh) & 1) + ((b >> sh) & 1);
              col = col * 4 + 2 * ((c >> sh) & 1) + ((d >> sh) & 1);
            }
            S[(size_t)row * sdim + col] += E(a, c) * std::conj(E(b, d));
          }
  }
  std::vector<double> out(2 * S.size());
  for (size_t i = 0; i < S.size(); ++i) {
    out[2 * i] = S[i].real();
    out[2 * i + 1] = S[i].imag();
  }
  return out;
}

int build_network(const tn_gate *gates_in, int n_gates, int n_qubits, const double *init,
                  const tn_target *target, int n_params, int dtype, Net &net) {
  if (n_qubits < 1 || n_qubits > 4096) { set_error("tn_build: n_qubits out of range"); return TN_EINVAL; }
  if (n_gates < 0 || (n_gates > 0 && !gates_in)) { set_error("tn_build: bad gate list"); return TN_EINVAL; }
  // channels given by Kraus operators become superoperator gates here
  std::vector<tn_gate> gate_copy(gates_in, gates_in + n_gates);
  std::vector<std::vector<double>> folded_store;
  for (int i = 0; i < n_gates; ++i) {
    tn_gate &g = gate_copy[i];
    if (g.kind != TN_KRAUS1 && g.kind != TN_KRAUS2) continue;
    if (!g.matrix || g.n_matrices < 1 || g.n_matrices > 4096) {
      set_error("tn_build: Kraus gate without operators at gate " + std::to_string(i));
      return TN_EINVAL;
    }
    folded_store.push_back(fold_kraus(g.matrix, g.n_matrices, g.kind == TN_KRAUS2));
    g.kind = g.kind == TN_KRAUS1 ? TN_SUPER1 : TN_SUPER2;
    g.matrix = folded_store.back().data();
  }
  const tn_gate *gates = gate_copy.data();
  if (!target) { set_error("tn_build: target is NULL"); return TN_EINVAL; }
  if (dtype != TN_C64 && dtype != TN_C128) { set_error("tn_build: bad dtype"); return TN_EINVAL; }
  if (n_params < 0) { set_error("tn_build: n_params < 0"); return TN_EINVAL; }
  const int mode = target->mode;
  if (mode != TN_AMPLITUDE && mode != TN_PROBABILITY && mode != TN_EXPECTATION) {
    set_error("tn_build: bad mode");
    return TN_EINVAL;
  }
  if ((mode == TN_EXPECTATION && !target->pauli) || (mode != TN_EXPECTATION && !target->bits)) {
    set_error("tn_build: target vector is NULL");
    return TN_EINVAL;
  }
  for (int q = 0; q < n_qubits; ++q) {
    int v = mode == TN_EXPECTATION ? target->pauli[q] : target->bits[q];
    int hi = mode == TN_EXPECTATION ? 3 : (mode == TN_PROBABILITY ? 2 : 1);
    if (v < 0 || v > hi) { set_error("tn_build: target entry out of range at qubit " + std::to_string(q)); return TN_EINVAL; }
  }
  bool all_unitary = true;
  for (int i = 0; i < n_gates; ++i) {
    const tn_gate &g = gates[i];
    if (g.kind < TN_H || g.kind > TN_SUPER2) { set_error("tn_build: bad gate kind at gate " + std::to_string(i)); return TN_EINVAL; }
    bool two = gate_is_2q(g.kind);
    if (g.q0 < 0 || g.q0 >= n_qubits || (two && (g.q1 < 0 || g.q1 >= n_qubits || g.q1 == g.q0)) || (!two && g.q1 != -1)) {
      set_error("tn_build: bad qubits at gate " + std::to_string(i));
      return TN_EINVAL;
    }
    if (g.param < -1 || g.param >= n_params || (g.param >= 0 && !gate_is_param(g.kind))) {
      set_error("tn_build: bad param index at gate " + std::to_string(i));
      return TN_EINVAL;
    }
    if ((g.kind == TN_U1 || g.kind == TN_U2 || gate_is_super(g.kind)) && !g.matrix) {
      set_error("tn_build: custom gate without matrix at gate " + std::to_string(i));
      return TN_EINVAL;
    }
    if (gate_is_super(g.kind) && mode == TN_AMPLITUDE) {
      set_error("tn_build: a channel (superoperator) needs a folded mode, at gate " + std::to_string(i));
      return TN_EINVAL;
    }
    if ((g.kind == TN_U1 || g.kind == TN_U2) && !is_unitary(gate_matrix(g, 0.0), g.kind == TN_U1 ? 2 : 4))
      all_unitary = false;
    if (gate_is_super(g.kind) && !is_trace_preserving(gate_matrix(g, 0.0), g.kind == TN_SUPER1 ? 1 : 2))
      all_unitary = false;
  }

  net = Net();
  net.n_qubits = n_qubits;
  net.mode = mode;
  net.dtype = dtype;
  net.n_params = n_params;
  const bool folded = mode != TN_AMPLITUDE;
  net.wire_bits = folded ? 2 : 1;

  // Backward light cone of the measured qubits: a gate none of whose qubits
  // is in the current support meets only trace vectors and, being unitary
  // (or a trace-preserving channel), contracts to trace vectors; it is
  // dropped. Kept gates add their qubits.
  // Consecutive diagonal gates commute, so a run of them is treated as one
  // layer: its gates are tested against the support at the run's late end.
  std::vector<char> keep(n_gates, 1), in_net(n_qubits, 1);
  if (folded && target->lightcone && all_unitary) {
    std::vector<char> sup(n_qubits, 0);
    for (int q = 0; q < n_qubits; ++q)
      sup[q] = mode == TN_EXPECTATION ? target->pauli[q] != 0 : target->bits[q] != 2;
    int i = n_gates - 1;
    while (i >= 0) {
      int j = i;
      if (gate_is_diagonal(gates[i]))
        while (j - 1 >= 0 && gate_is_diagonal(gates[j - 1])) --j;
      std::vector<int> grow;
      for (int k = i; k >= j; --k) {
        const tn_gate &g = gates[k];
        bool touch = sup[g.q0] || (g.q1 >= 0 && sup[g.q1]);
        keep[k] = touch;
        if (touch) {
          grow.push_back(g.q0);
          if (g.q1 >= 0) grow.push_back(g.q1);
        }
      }
      for (int q : grow) sup[q] = 1;
      i = j - 1;
    }
    in_net = sup;
  }

  Builder B(net);
  std::vector<int> cur(n_qubits, -1);
  for (int q = 0; q < n_qubits; ++q) {
    if (!in_net[q]) continue;
    cd p0 = init ? cd(init[4 * q], init[4 * q + 1]) : cd(1, 0);
    cd p1 = init ? cd(init[4 * q + 2], init[4 * q + 3]) : cd(0, 0);
    Mat v = folded ? Mat{p0 * std::conj(p0), p0 * std::conj(p1), p1 * std::conj(p0), p1 * std::conj(p1)} : Mat{p0, p1};
    int w = B.new_wire();
    B.add_leaf({w}, B.add_const(v));
    cur[q] = w;
  }
  // diagonal mode: a gate diagonal in the computational basis keeps its
  // wires (input = output) and becomes a tensor of its diagonal on them;
  // those wires become hyperedges held by more than two tensors
  const bool diag_mode = target->diagonal != 0;
  for (int i = 0; i < n_gates; ++i) {
    if (!keep[i]) continue;
    const tn_gate &g = gates[i];
    if (diag_mode && gate_is_diagonal(g)) {
      const bool two = gate_is_2q(g.kind);
      int src = g.param >= 0 ? -B.add_ptensor(g.kind, g.param, g.coeff, folded, 1) - 1
                             : B.add_const(diag_entries(gate_matrix(g, g.coeff), two, folded));
      if (two) B.add_leaf({cur[g.q0], cur[g.q1]}, src);
      else B.add_leaf({cur[g.q0]}, src);
      continue;
    }
    int src;
    if (g.param >= 0) {
      src = -B.add_ptensor(g.kind, g.param, g.coeff, folded, 0) - 1;
    } else {
      Mat U = gate_matrix(g, g.coeff);
      bool two = gate_is_2q(g.kind);
      src = B.add_const(gate_is_super(g.kind) ? U : (folded ? (two ? superop_2q(U) : superop_1q(U)) : U));
    }
    if (g.q1 < 0) {
      int w = B.new_wire();
      B.add_leaf({w, cur[g.q0]}, src);
      cur[g.q0] = w;
    } else {
      int w0 = B.new_wire(), w1 = B.new_wire();
      B.add_leaf({w0, w1, cur[g.q0], cur[g.q1]}, src);
      cur[g.q0] = w0;
      cur[g.q1] = w1;
    }
  }
  for (int q = 0; q < n_qubits; ++q) {
    if (!in_net[q]) continue;
    Mat v;
    if (mode == TN_AMPLITUDE) {
      v = target->bits[q] ? Mat{0, 1} : Mat{1, 0};
    } else if (mode == TN_PROBABILITY) {
      int b = target->bits[q];
      v = b == 0 ? Mat{1, 0, 0, 0} : (b == 1 ? Mat{0, 0, 0, 1} : Mat{1, 0, 0, 1});
    } else {
      Mat P = pauli(target->pauli[q]);
      v = {P[0], P[2], P[1], P[3]};  // entry 2a+b = P_ba
    }
    B.add_leaf({cur[q]}, B.add_const(v));
  }
  return TN_OK;
}

}  // namespace qtn
