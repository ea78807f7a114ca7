"""Gate matrices for the oracle (test infrastructure; see package docstring).

Plain definitions of the one- and two-qubit unitaries the circuits use.
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
PAULI = {0: I2, 1: X, 2: Y, 3: Z, "I": I2, "X": X, "Y": Y, "Z": Z}


def rot(P, theta):
    """exp(-i theta P / 2) for a Pauli matrix P (P @ P = I)."""
    return np.cos(theta / 2) * np.eye(P.shape[0], dtype=np.complex128) - 1j * np.sin(theta / 2) * P


def zz(theta):
    """exp(-i theta Z(x)Z / 2): a diagonal 4x4 matrix."""
    return rot(np.kron(Z, Z), theta)


CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)


def random_unitary_matrix(dim, seed):
    import workloads
    return np.array(workloads.random_unitary(dim, seed), dtype=np.complex128)


def gate_matrix(kind, theta=0.0, matrix_seed=0, matrix=None):
    """Matrix of a gate given by its kind name (circuit description)."""
    if matrix is not None:
        return np.asarray(matrix, dtype=np.complex128)
    if kind == "H":
        return H
    if kind == "X":
        return X
    if kind == "Y":
        return Y
    if kind == "Z":
        return Z
    if kind == "RX":
        return rot(X, theta)
    if kind == "RY":
        return rot(Y, theta)
    if kind == "RZ":
        return rot(Z, theta)
    if kind == "ZZ":
        return zz(theta)
    if kind == "CNOT":
        return CNOT
    if kind == "CZ":
        return CZ
    if kind == "U1":
        return random_unitary_matrix(2, matrix_seed)
    if kind == "U2":
        return random_unitary_matrix(4, matrix_seed)
    raise ValueError(kind)


def qaoa_gate_list(n, edges, gammas, betas):
    """QAOA Max-Cut circuit (Sec. QAOA / Max-Cut) as (kind, q0, q1, theta) tuples.

    H on every qubit, then per layer k: exp(-i gamma_k Z_u Z_v) per edge
    (ZZ(2 gamma_k)) and exp(-i beta_k X) per qubit (R_X(2 beta_k)).
    """
    gl = [("H", q, -1, 0.0) for q in range(n)]
    for g, b in zip(gammas, betas):
        gl += [("ZZ", u, v, 2.0 * g) for (u, v) in edges]
        gl += [("RX", q, -1, 2.0 * b) for q in range(n)]
    return gl
