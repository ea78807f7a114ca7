"""Noise channels given by their Kraus operators (TN_KRAUS1 / TN_KRAUS2 gates).

A channel rho -> sum_k E_k rho E_k^dagger becomes one tensor of the folded
network, the same way a unitary gate U becomes U (x) conj(U) (the paper's
treatment of noise via Kraus operators). tn_build folds the operators into
the superoperator; these helpers give the operators of common channels and
the gate tuples for `qtn.Network`.
"""
import numpy as np


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
    """Gate tuple of the channel with Kraus operators `kraus` (2x2, or 4x4 with
    basis index 2 x_q0 + x_q1) on qubit q0 (and q1)."""
    return ("KRAUS1" if q1 < 0 else "KRAUS2", q0, q1, -1, 0.0, [np.asarray(k, dtype=np.complex128) for k in kraus])
