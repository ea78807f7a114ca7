"""Plain FP64 tensor-network contractor (test infrastructure).

Follows Sec. Preliminaries of the paper:
  * a circuit becomes a closed network whose nodes are initial states, gates
    and measurements, with the circuit's own connectivity;
  * in the folded (density-matrix) form every wire has dimension 4 and
    carries the vectorised density matrix [rho00, rho01, rho10, rho11], i.e.
    index 2a+b holds rho_ab;
  * a gate U acting as rho -> U rho U^dagger becomes the superoperator tensor
    with entries U_ac * conj(U_bd) from input (c,d) to output (a,b); a
    two-qubit gate has four wires ordered (q0 out, q1 out, q0 in, q1 in);
  * a measurement of Pauli P is the vector M[2a+b] = P_ba, so that
    sum_k M_k rho_k = Tr(P rho); P = I gives the trace vector [1,0,0,1];
  * the network is contracted pairwise, eq. (1): all indices shared by the two
    tensors are summed at once (numpy.tensordot), until one scalar is left;
    scalars of disconnected pieces are multiplied.
The unfolded (amplitude) network uses dimension-2 wires, gate matrices U and
output row vectors <x|. The doubled network keeps a ket layer (U) and a bra
layer (conj U) joined by the measured operator; it is a cross-check of the
folding convention.
"""
import itertools

import numpy as np

from . import gates


class Network:
    """Tensors with integer wire labels per axis; each label appears twice."""

    def __init__(self):
        self.tensors = []
        self.legs = []
        self._next = 0

    def wire(self):
        self._next += 1
        return self._next - 1

    def add(self, t, legs):
        t = np.asarray(t, dtype=np.complex128)
        assert t.ndim == len(legs)
        self.tensors.append(t)
        self.legs.append(list(legs))

    def check_closed(self):
        from collections import Counter
        c = Counter(w for legs in self.legs for w in legs)
        assert all(v == 2 for v in c.values()), "every wire must join exactly two tensor axes"


# --- superoperator tensors ------------------------------------------------

def vec_density(psi):
    """Vectorised |psi><psi| of one qubit: entry 2a+b = psi_a conj(psi_b)."""
    psi = np.asarray(psi, dtype=np.complex128)
    return np.array([psi[a] * np.conj(psi[b]) for a in range(2) for b in range(2)])


def superop_1q(U):
    """4x4 tensor S[(ab),(cd)] = U_ac conj(U_bd); axes (out, in)."""
    S = np.zeros((4, 4), dtype=np.complex128)
    for a, b, c, d in itertools.product(range(2), repeat=4):
        S[2 * a + b, 2 * c + d] = U[a, c] * np.conj(U[b, d])
    return S


def superop_2q(U):
    """4x4x4x4 tensor with axes (q0 out, q1 out, q0 in, q1 in).

    S[(a0 b0),(a1 b1),(c0 d0),(c1 d1)] = U[(a0 a1),(c0 c1)] conj(U[(b0 b1),(d0 d1)]).
    """
    S = np.zeros((4, 4, 4, 4), dtype=np.complex128)
    for a0, b0, a1, b1, c0, d0, c1, d1 in itertools.product(range(2), repeat=8):
        S[2 * a0 + b0, 2 * a1 + b1, 2 * c0 + d0, 2 * c1 + d1] = (
            U[2 * a0 + a1, 2 * c0 + c1] * np.conj(U[2 * b0 + b1, 2 * d0 + d1]))
    return S


def measure_vec(P):
    """M[2a+b] = P_ba, so that sum_k M_k vec(rho)_k = Tr(P rho)."""
    return np.array([P[b, a] for a in range(2) for b in range(2)], dtype=np.complex128)


PROJ = {0: np.array([[1, 0], [0, 0]], dtype=np.complex128),
        1: np.array([[0, 0], [0, 1]], dtype=np.complex128),
        2: np.eye(2, dtype=np.complex128)}


# --- light cone -------------------------------------------------------------

DIAGONAL = {"Z", "RZ", "ZZ", "CZ"}


def light_cone(n, gate_list, support):
    """Gates that can influence observables on `support` (a set of qubits).

    Walking backwards, a gate with no qubit in the current support is dropped
    (for a unitary gate its superoperator meets trace vectors only and
    contracts to trace vectors); a kept two-qubit gate adds both qubits.
    Gates diagonal in the computational basis commute, so a run of them is
    one layer: each is tested against the support at the run's late end.
    Returns (kept gates in circuit order, final support).
    """
    sup = set(support)
    kept = []
    i = len(gate_list) - 1
    while i >= 0:
        j = i
        if gate_list[i][0] in DIAGONAL:
            while j - 1 >= 0 and gate_list[j - 1][0] in DIAGONAL:
                j -= 1
        grow = set()
        for g in reversed(gate_list[j:i + 1]):
            qs = [g[1]] + ([g[2]] if g[2] >= 0 else [])
            if any(q in sup for q in qs):
                kept.append(g)
                grow.update(qs)
        sup |= grow
        i = j - 1
    return kept[::-1], sup


# --- network construction ----------------------------------------------------

def _init_vectors(n, init):
    if init is None:
        return [np.array([1.0, 0.0], dtype=np.complex128)] * n
    return [np.asarray(v, dtype=np.complex128) for v in init]


def folded_network(n, gate_list, meas_ops, init=None, qubits=None):
    """Closed folded network: rho~_q -> superoperators -> measurement vectors.

    meas_ops[q] is the 2x2 operator measured on qubit q (identity = trace).
    Only qubits in `qubits` (default all) get boundary tensors.
    """
    qubits = sorted(range(n) if qubits is None else qubits)
    init = _init_vectors(n, init)
    net = Network()
    cur = {}
    for q in qubits:
        w = net.wire()
        net.add(vec_density(init[q]), [w])
        cur[q] = w
    for g in gate_list:
        kind, q0, q1, theta = g[:4]
        mseed = g[4] if len(g) > 4 else 0
        U = gates.gate_matrix(kind, theta, mseed)
        if q1 < 0:
            w = net.wire()
            net.add(superop_1q(U), [w, cur[q0]])
            cur[q0] = w
        else:
            w0, w1 = net.wire(), net.wire()
            net.add(superop_2q(U), [w0, w1, cur[q0], cur[q1]])
            cur[q0], cur[q1] = w0, w1
    for q in qubits:
        net.add(measure_vec(meas_ops[q]), [cur[q]])
    net.check_closed()
    return net


def amplitude_network(n, gate_list, bits, init=None):
    """Closed dimension-2 network for <bits| C |psi0>."""
    init = _init_vectors(n, init)
    net = Network()
    cur = {}
    for q in range(n):
        w = net.wire()
        net.add(init[q], [w])
        cur[q] = w
    for g in gate_list:
        kind, q0, q1, theta = g[:4]
        mseed = g[4] if len(g) > 4 else 0
        U = gates.gate_matrix(kind, theta, mseed)
        if q1 < 0:
            w = net.wire()
            net.add(U, [w, cur[q0]])
            cur[q0] = w
        else:
            w0, w1 = net.wire(), net.wire()
            net.add(U.reshape(2, 2, 2, 2), [w0, w1, cur[q0], cur[q1]])
            cur[q0], cur[q1] = w0, w1
    for q in range(n):
        e = np.zeros(2, dtype=np.complex128)
        e[bits[q]] = 1.0
        net.add(e, [cur[q]])
    net.check_closed()
    return net


def doubled_network(n, gate_list, meas_ops, init=None):
    """<psi| (x)_q P_q |psi> as a ket layer, a bra layer and 2x2 operators."""
    init = _init_vectors(n, init)
    net = Network()
    ket, bra = {}, {}
    for q in range(n):
        wk, wb = net.wire(), net.wire()
        net.add(init[q], [wk])
        net.add(np.conj(init[q]), [wb])
        ket[q], bra[q] = wk, wb
    for g in gate_list:
        kind, q0, q1, theta = g[:4]
        mseed = g[4] if len(g) > 4 else 0
        U = gates.gate_matrix(kind, theta, mseed)
        for layer, f in ((ket, lambda m: m), (bra, np.conj)):
            if q1 < 0:
                w = net.wire()
                net.add(f(U), [w, layer[q0]])
                layer[q0] = w
            else:
                w0, w1 = net.wire(), net.wire()
                net.add(f(U).reshape(2, 2, 2, 2), [w0, w1, layer[q0], layer[q1]])
                layer[q0], layer[q1] = w0, w1
    for q in range(n):
        # <psi|P|psi> = sum_ab conj(psi_a) P_ab psi_b : bra index a, ket index b
        net.add(meas_ops[q], [bra[q], ket[q]])
    net.check_closed()
    return net


# --- contraction -------------------------------------------------------------

def contract_pair(A, la, B, lb):
    """Eq. (1): sum over every label shared by A and B; result legs = free(A) ++ free(B)."""
    shared = [w for w in la if w in lb]
    ia = [la.index(w) for w in shared]
    ib = [lb.index(w) for w in shared]
    C = np.tensordot(A, B, axes=(ia, ib))
    lc = [w for w in la if w not in shared] + [w for w in lb if w not in shared]
    return C, lc


def contract(net, order=None):
    """Contract the closed network to a complex scalar.

    order: optional sequence of wire labels; each wire joining two different
    tensors merges them (wires already inside one tensor are skipped).
    Without an order a greedy rule picks the pair with the smallest result.
    """
    ts = list(net.tensors)
    ls = [list(l) for l in net.legs]
    alive = list(range(len(ts)))

    def owner(w):
        return [i for i in alive if w in ls[i]]

    def merge(i, j):
        C, lc = contract_pair(ts[i], ls[i], ts[j], ls[j])
        ts.append(C)
        ls.append(lc)
        alive.remove(i)
        alive.remove(j)
        alive.append(len(ts) - 1)

    if order is not None:
        for w in order:
            o = owner(w)
            if len(o) == 2:
                merge(o[0], o[1])
    while True:
        best = None
        for a in range(len(alive)):
            for b in range(a + 1, len(alive)):
                i, j = alive[a], alive[b]
                sh = set(ls[i]) & set(ls[j])
                if not sh:
                    continue
                size = ts[i].size * ts[j].size // (np.prod([ts[i].shape[ls[i].index(w)] for w in sh]) ** 2)
                if best is None or size < best[0]:
                    best = (size, i, j)
        if best is None:
            break
        merge(best[1], best[2])
    val = np.complex128(1.0)
    for i in alive:
        assert ts[i].ndim == 0
        val = val * ts[i][()]
    return complex(val)


# --- user-level quantities -----------------------------------------------------

def expectation(n, gate_list, pauli, init=None, lightcone=False):
    """<psi|P|psi> for a Pauli string (codes 0=I 1=X 2=Y 3=Z), folded network."""
    qubits = None
    gl = gate_list
    if lightcone:
        gl, qubits = light_cone(n, gate_list, [q for q in range(n) if pauli[q]])
    ops = [gates.PAULI[c] for c in pauli]
    return contract(folded_network(n, gl, ops, init, qubits))


def probability(n, gate_list, bits, init=None):
    """Tr(Pi rho_out) with Pi = (x)_q Pi_q; bits[q] in {0, 1} projects, 2 traces."""
    ops = [PROJ[b] for b in bits]
    return contract(folded_network(n, gate_list, ops, init))


def amplitude(n, gate_list, bits, init=None):
    return contract(amplitude_network(n, gate_list, bits, init))


def qaoa_zz(n, edges, gammas, betas, lightcone=True):
    """<Z_u Z_v> per edge, one folded network per edge."""
    gl = gates.qaoa_gate_list(n, edges, gammas, betas)
    plus = [np.array([1.0, 1.0]) / np.sqrt(2.0)] * n
    gl = gl[n:]  # the H layer is folded into the |+> boundary vectors
    out = []
    for (u, v) in edges:
        pauli = [0] * n
        pauli[u] = pauli[v] = 3
        out.append(expectation(n, gl, pauli, init=plus, lightcone=lightcone).real)
    return np.array(out)
