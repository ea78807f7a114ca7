"""Pins of the density-matrix oracle (noisy circuits) against facts fixed by
mathematics: unitary evolution agrees with the state-vector oracle,
standard channels act on the Bloch vector as their closed forms say,
trace-preserving channels keep Tr rho = 1, and a projection returns the Born
probability."""
import numpy as np
import pytest

import workloads
from oracle import density, gates, statevector

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]])
Z = np.diag([1.0, -1.0]).astype(np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def _dep(p):
    return [np.sqrt(1 - 0.75 * p) * I2, np.sqrt(p / 4) * X, np.sqrt(p / 4) * Y, np.sqrt(p / 4) * Z]


def _plus_rho(n):
    return density.pure(statevector.product_state([[1 / np.sqrt(2), 1 / np.sqrt(2)]] * n))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_unitary_circuits_match_statevector(seed):
    n = 4
    desc = workloads.random_circuit(n, 20, seed)
    gl = [(k, q0, q1, th, ms) for k, q0, q1, th, ms in desc]
    psi = statevector.run(n, gl)
    ops = [([gates.gate_matrix(k, th, ms)], [q0] if q1 < 0 else [q0, q1]) for k, q0, q1, th, ms in gl]
    rho = density.run(n, ops, density.pure(statevector.zero_state(n)))
    rng = np.random.default_rng(seed)
    for _ in range(5):
        pa = list(rng.integers(0, 4, size=n))
        np.testing.assert_allclose(density.expect_pauli(rho, pa), statevector.expect_pauli(psi, pa), atol=1e-13)
        bits = list(rng.integers(0, 3, size=n))
        prob = np.abs(psi) ** 2
        for q in reversed(range(n)):
            prob = prob.sum(axis=q) if bits[q] == 2 else np.take(prob, bits[q], axis=q)
        np.testing.assert_allclose(density.probability(rho, bits).real, float(prob), atol=1e-13)


def test_depolarizing_shrinks_the_bloch_vector():
    for p in (0.0, 0.1, 0.37, 1.0):
        rho = density.apply_channel(_plus_rho(1), _dep(p), [0])
        np.testing.assert_allclose(density.expect_pauli(rho, [1]), 1 - p, atol=1e-15)
        np.testing.assert_allclose(density.expect_pauli(rho, [0]), 1.0, atol=1e-15)


def test_amplitude_damping_closed_form():
    g = 0.3
    K = [np.array([[1, 0], [0, np.sqrt(1 - g)]]), np.array([[0, np.sqrt(g)], [0, 0]])]
    one = density.pure(np.array([0.0, 1.0]))
    rho = density.apply_channel(one, K, [0])
    np.testing.assert_allclose(density.probability(rho, [0]).real, g, atol=1e-15)
    rho = density.apply_channel(_plus_rho(1), K, [0])
    np.testing.assert_allclose(density.expect_pauli(rho, [1]).real, np.sqrt(1 - g), atol=1e-15)
    np.testing.assert_allclose(density.expect_pauli(rho, [3]).real, g, atol=1e-15)


def test_dephasing_and_trace_preservation():
    p = 0.2
    K = [np.sqrt(1 - p) * I2, np.sqrt(p) * Z]
    rho = density.apply_channel(_plus_rho(2), K, [1])
    np.testing.assert_allclose(density.expect_pauli(rho, [1, 1]).real, 1 - 2 * p, atol=1e-15)
    # a random channel from a Haar isometry (4 Kraus operators on 2 qubits) keeps the trace
    rng = np.random.default_rng(5)
    z = rng.normal(size=(16, 4)) + 1j * rng.normal(size=(16, 4))
    V, _ = np.linalg.qr(z)  # 16 x 4 isometry
    kraus = [V[4 * k:4 * (k + 1), :] for k in range(4)]
    rho = density.apply_channel(_plus_rho(3), kraus, [0, 2])
    np.testing.assert_allclose(density.probability(rho, [2, 2, 2]).real, 1.0, atol=1e-14)


def test_projection_gives_the_born_probability_and_product_channels_factor():
    n = 3
    gl = [("H", 0, -1, 0.0), ("CNOT", 0, 1, 0.0), ("RY", 2, -1, 0.9), ("CZ", 1, 2, 0.0)]
    psi = statevector.run(n, gl)
    ops = [([gates.gate_matrix(k, t)], [a] if b < 0 else [a, b]) for k, a, b, t in gl]
    rho = density.run(n, ops, density.pure(statevector.zero_state(n)))
    proj = density.apply_channel(rho, [np.diag([0.0, 1.0])], [1])
    np.testing.assert_allclose(density.probability(proj, [2, 2, 2]).real, np.sum(np.abs(psi[:, 1, :]) ** 2),
                               atol=1e-14)
    # depolarizing on both qubits of a pair = the two-qubit channel with product Kraus operators
    a = density.apply_channel(density.apply_channel(rho, _dep(0.2), [0]), _dep(0.3), [2])
    prod = [np.kron(E, F) for E in _dep(0.2) for F in _dep(0.3)]
    b = density.apply_channel(rho, prod, [0, 2])
    np.testing.assert_allclose(a, b, atol=1e-14)
