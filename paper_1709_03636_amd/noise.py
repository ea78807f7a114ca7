"""Noise channels as folded superoperators (TN_SUPER1 / TN_SUPER2 gates).

A channel rho -> sum_k E_k rho E_k^dagger becomes one tensor of the folded
network, the same way a unitary gate U becomes U (x) conj(U): the paper's
treatment of noise via Kraus operators. These helpers build the superoperator
in the layout the C ABI documents (output wires first, each wire value
2a + b for rho_ab) and return gate tuples for `qtn.Network`.
"""
import numpy as np


def superop(kraus):
    """Folded superoperator of the Kraus operators `kraus` (2x2 or 4x4 each):
    S[(a, b), (c, d)] = sum_k E_k[a, c] conj(E_k[b, d]) with a, b, c, d the
    output-ket, output-bra, input-ket and input-bra indices; for two qubits
    each of them splits into (qubit q0 bit, qubit q1 bit) and the wire order
    is (q0 out, q1 out, q0 in, q1 in)."""
    ks = [np.asarray(k, dtype=np.complex128) for k in kraus]
    dim = ks[0].shape[0]
    S = sum(np.einsum("ac,bd->abcd", k, k.conj()) for k in ks)  # [a, b, c, d]
    if dim == 2:
        return S.reshape(4, 4)  # (2a+b, 2c+d)
    S = S.reshape(2, 2, 2, 2, 2, 2, 2, 2)  # a0 a1 b0 b1 c0 c1 d0 d1
    return S.transpose(0, 2, 1, 3, 4, 6, 5, 7).reshape(16, 16)  # (a0 b0 a1 b1), (c0 d0 c1 d1)


def depolarizing(p):
    """rho -> (1 - p) rho + p I/2: Kraus sqrt(1 - 3p/4) I, sqrt(p/4) X, Y, Z."""
    I = np.eye(2)
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1.0, -1.0])
    return [np.sqrt(1 - 0.75 * p) * I, np.sqrt(p / 4) * X, np.sqrt(p / 4) * Y, np.sqrt(p / 4) * Z]


def amplitude_damping(g):
    """|1> decays to |0> with probability g."""
    return [np.array([[1, 0], [0, np.sqrt(1 - g)]]), np.array([[0, np.sqrt(g)], [0, 0]])]


def dephasing(p):
    """rho -> (1 - p) rho + p Z rho Z."""
    return [np.sqrt(1 - p) * np.eye(2), np.sqrt(p) * np.diag([1.0, -1.0])]


def channel_gate(kraus, q0, q1=-1):
    """Gate tuple of the channel on qubit q0 (and q1 for a two-qubit channel)."""
    S = superop(kraus)
    return ("SUPER1" if q1 < 0 else "SUPER2", q0, q1, -1, 0.0, S)
