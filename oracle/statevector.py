"""Brute-force 2^N state-vector simulation (test infrastructure).

The plain definition of what a circuit computes (Sec. Introduction: given a
circuit and an initial state, determine output amplitudes, probabilities and
expectation values <psi|M|psi> of Pauli strings, Sec. "Estimating the answer
string"). Qubit q is axis q of a (2,)*n array, so qubit 0 is the most
significant bit of the flat basis index.
"""
import numpy as np

from . import gates


def zero_state(n):
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def product_state(vectors):
    """Tensor product of one 2-vector per qubit."""
    psi = np.array(1.0 + 0j)
    for v in vectors:
        psi = np.multiply.outer(psi, np.asarray(v, dtype=np.complex128))
    return psi


def apply_1q(psi, U, q):
    psi = np.tensordot(U, psi, axes=([1], [q]))
    return np.moveaxis(psi, 0, q)


def apply_2q(psi, U, q0, q1):
    U4 = U.reshape(2, 2, 2, 2)
    psi = np.tensordot(U4, psi, axes=([2, 3], [q0, q1]))
    return np.moveaxis(psi, [0, 1], [q0, q1])


def run(n, gate_list, psi0=None):
    """Apply (kind, q0, q1, theta[, matrix_seed]) gates in order."""
    psi = zero_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128).reshape((2,) * n)
    for g in gate_list:
        kind, q0, q1, theta = g[:4]
        mseed = g[4] if len(g) > 4 else 0
        U = gates.gate_matrix(kind, theta, mseed)
        psi = apply_1q(psi, U, q0) if q1 < 0 else apply_2q(psi, U, q0, q1)
    return psi


def expect_pauli(psi, pauli):
    """<psi| P_0 (x) ... (x) P_{n-1} |psi> for pauli codes 0=I 1=X 2=Y 3=Z."""
    phi = psi
    for q, c in enumerate(pauli):
        if c:
            phi = apply_1q(phi, gates.PAULI[c], q)
    return np.vdot(psi.ravel(), phi.ravel())


def qaoa_state(n, edges, gammas, betas):
    return run(n, gates.qaoa_gate_list(n, edges, gammas, betas))


def qaoa_zz(n, edges, gammas, betas):
    """<Z_u Z_v> for every edge, from one state vector."""
    prob = np.abs(qaoa_state(n, edges, gammas, betas)) ** 2
    sign = np.array([1.0, -1.0])
    out = []
    for (u, v) in edges:
        marg = np.moveaxis(prob, [u, v], [0, 1]).reshape(2, 2, -1).sum(axis=2)
        out.append(float(sign @ marg @ sign))
    return np.array(out)


def qaoa_cost(n, edges, gammas, betas):
    """<C> = sum over edges of (1 - <Z_u Z_v>)/2 (Sec. QAOA / Max-Cut)."""
    return float(np.sum((1.0 - qaoa_zz(n, edges, gammas, betas)) / 2.0))


def qaoa_edge_lightcone_circuit(n, edges, gammas, betas, edge, with_index=False):
    """(qubit count, gate list, (u', v')) of the backward light cone of one edge.

    Gates outside the light cone of Z_u Z_v do not change <Z_u Z_v>
    (unitarity); the kept gates act only on the support, relabelled 0..m-1.
    with_index also returns each kept gate's position in the full QAOA gate
    list (H layer first, then per layer |E| ZZ gates and n X rotations).
    """
    from .tensornet import light_cone
    u, v = edge
    gl = gates.qaoa_gate_list(n, edges, gammas, betas)
    tagged = [g + (i,) for i, g in enumerate(gl)]
    kept, sup = light_cone(n, tagged, {u, v})
    qubits = sorted(sup)
    idx = {q: i for i, q in enumerate(qubits)}
    sub = [(g[0], idx[g[1]], idx[g[2]] if g[2] >= 0 else -1, g[3]) for g in kept]
    if with_index:
        return len(qubits), sub, (idx[u], idx[v]), [g[4] for g in kept]
    return len(qubits), sub, (idx[u], idx[v])


def zz_of(m, gate_list, uv):
    prob = np.abs(run(m, gate_list)) ** 2
    marg = np.moveaxis(prob, list(uv), [0, 1]).reshape(2, 2, -1).sum(axis=2)
    sign = np.array([1.0, -1.0])
    return float(sign @ marg @ sign)


def qaoa_zz_edge(n, edges, gammas, betas, edge):
    """<Z_u Z_v> of one edge from a state vector over its light cone only."""
    m, sub, uv = qaoa_edge_lightcone_circuit(n, edges, gammas, betas, edge)
    return zz_of(m, sub, uv)
