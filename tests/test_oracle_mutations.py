"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin fails.

Each mutation replaces one oracle function with a subtly wrong version (a
dropped conjugate, a transposed operand, a lost term); the pins of
test_oracle_pins must then fail. This shows the pins constrain the oracle.
"""
import itertools

import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import closed_form, tensornet


def _any_pin_fails(checks):
    for chk in checks:
        try:
            chk()
        except AssertionError:
            return True
    return False


TN_CHECKS = [
    pins.test_printed_initial_state,
    lambda: pins.test_printed_pauli_superoperators("Y", pins.gates.Y),
    pins.test_printed_cnot_nonzeros,
    lambda: pins.test_printed_measurement_vectors("M_Y", pins.gates.Y),
    pins.test_superop_1q_is_conjugation,
    pins.test_superop_2q_is_conjugation,
    lambda: pins.test_tn_expectation_matches_statevector(1),
    lambda: pins.test_tn_amplitude_and_probability(0),
    pins.test_tn_qaoa_matches_statevector_p2,
]


def _superop_1q_no_conj(U):
    S = np.zeros((4, 4), dtype=np.complex128)
    for a, b, c, d in itertools.product(range(2), repeat=4):
        S[2 * a + b, 2 * c + d] = U[a, c] * U[b, d]
    return S


def _superop_1q_transposed(U):
    S = np.zeros((4, 4), dtype=np.complex128)
    for a, b, c, d in itertools.product(range(2), repeat=4):
        S[2 * a + b, 2 * c + d] = U[c, a] * np.conj(U[d, b])
    return S


def _superop_2q_swapped_wires(U):
    return np.transpose(tensornet.__dict__["_orig_superop_2q"](U), (1, 0, 3, 2))


def _measure_vec_transposed(P):
    return np.array([P[a, b] for a in range(2) for b in range(2)], dtype=np.complex128)


def _vec_density_no_conj(psi):
    psi = np.asarray(psi, dtype=np.complex128)
    return np.array([psi[a] * psi[b] for a in range(2) for b in range(2)])


@pytest.mark.parametrize("name,bad", [
    ("superop_1q", _superop_1q_no_conj),
    ("superop_1q", _superop_1q_transposed),
    ("superop_2q", _superop_2q_swapped_wires),
    ("measure_vec", _measure_vec_transposed),
    ("vec_density", _vec_density_no_conj),
])
def test_tensor_mutations_are_caught(monkeypatch, name, bad):
    monkeypatch.setitem(tensornet.__dict__, "_orig_superop_2q", tensornet.superop_2q)
    monkeypatch.setattr(tensornet, name, bad)
    assert _any_pin_fails(TN_CHECKS), f"mutation of {name} not caught"


def test_closed_form_dropped_triangle_term_is_caught(monkeypatch):
    orig = closed_form.zz_p1

    def no_triangles(n, edges, gamma, beta):
        c2g, s2g, s4b, s2b = np.cos(2 * gamma), np.sin(2 * gamma), np.sin(4 * beta), np.sin(2 * beta)
        nb = closed_form._graph_facts(n, edges)
        return np.array([0.5 * s4b * s2g * (c2g ** (len(nb[u]) - 1) + c2g ** (len(nb[v]) - 1)) for u, v in edges])

    monkeypatch.setattr(closed_form, "zz_p1", no_triangles)
    checks = [lambda: pins.test_closed_form_matches_statevector(3, 12, 0),
              lambda: pins.test_closed_form_matches_statevector(4, 10, 0)]
    assert _any_pin_fails(checks)
    monkeypatch.setattr(closed_form, "zz_p1", orig)


def test_closed_form_sign_error_is_caught(monkeypatch):
    orig = closed_form.zz_p1
    monkeypatch.setattr(closed_form, "zz_p1", lambda n, e, g, b: orig(n, e, -g, b))
    assert _any_pin_fails([pins.test_triangle_free_3regular_optimum_statevector,
                           lambda: pins.test_closed_form_matches_statevector(3, 12, 1)])
