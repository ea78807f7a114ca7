"""Density-matrix simulation in FP64 (test infrastructure).

The plain definition of a noisy circuit: rho evolves as rho -> U rho U^dagger
for a gate and rho -> sum_k E_k rho E_k^dagger for a channel given by its
Kraus operators (the paper's noise model); measured quantities are
Tr(P rho) and Tr(Pi rho). rho is an array of shape (2,)*n + (2,)*n (ket axes
then bra axes, qubit 0 first).
"""
import numpy as np


def pure(psi):
    psi = np.asarray(psi, dtype=np.complex128)
    return np.multiply.outer(psi, psi.conj())


def _apply_op(rho, E, qubits, n):
    """E rho E^dagger for an operator E on `qubits` (E indexed (out..., in...))."""
    k = len(qubits)
    E = np.asarray(E, dtype=np.complex128).reshape((2,) * (2 * k))
    # ket side
    rho = np.tensordot(E, rho, axes=(list(range(k, 2 * k)), list(qubits)))
    rho = np.moveaxis(rho, list(range(k)), list(qubits))
    # bra side: rho E^dagger, i.e. contract conj(E) on the bra axes
    bra = [n + q for q in qubits]
    rho = np.tensordot(E.conj(), rho, axes=(list(range(k, 2 * k)), bra))
    return np.moveaxis(rho, list(range(k)), bra)


def apply_channel(rho, kraus, qubits):
    n = rho.ndim // 2
    return sum(_apply_op(rho, E, qubits, n) for E in kraus)


def run(n, ops, rho0):
    """ops: list of (kraus_list, qubits); a unitary gate is a one-element list."""
    rho = rho0
    for kraus, qubits in ops:
        rho = apply_channel(rho, kraus, qubits)
    return rho


def trace_with(rho, local_ops):
    """Tr((O_0 (x) ... (x) O_{n-1}) rho) for one 2x2 operator per qubit."""
    n = rho.ndim // 2
    r = rho
    for q in range(n):
        O = np.asarray(local_ops[q], dtype=np.complex128)
        # contract O[b, a] with rho[a(ket q), b(bra q)] at the leading ket/bra axes
        r = np.tensordot(r, O, axes=([0, n - q], [1, 0]))
    return complex(r)


def expect_pauli(rho, pauli):
    P = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]
    return trace_with(rho, [P[c] for c in pauli])


def probability(rho, bits):
    """Tr(Pi rho), Pi = projector |b><b| on qubits with b in {0, 1}, identity for 2."""
    M = [np.diag([1.0, 0.0]), np.diag([0.0, 1.0]), np.eye(2)]
    return trace_with(rho, [M[b] for b in bits])
