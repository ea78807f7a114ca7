"""Pins of the FP64 oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself or with the HIP path: the
expected values are the paper's printed tensors (tests/golden), textbook
identities, brute-force state vectors on tiny inputs, a published p=1 QAOA
optimum, closed forms and exact special cases.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import closed_form, gates, gradients, statevector, tensornet

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _rand_rho(seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    r = a @ a.conj().T
    return r / np.trace(r)


def _vec(rho):
    return np.array([rho[0, 0], rho[0, 1], rho[1, 0], rho[1, 1]])


# --- the paper's printed tensors -------------------------------------------------

def test_printed_initial_state():
    g = _gold("paper_tensors.json")["rho0"]
    got = tensornet.vec_density([1.0, 0.0])
    np.testing.assert_array_equal(got, np.array(g["re"]) + 1j * np.array(g["im"]))


@pytest.mark.parametrize("name,U", [("X", gates.X), ("Y", gates.Y)])
def test_printed_pauli_superoperators(name, U):
    g = _gold("paper_tensors.json")[name]
    np.testing.assert_allclose(tensornet.superop_1q(U), np.array(g["re"]), atol=0)


def test_printed_Z_is_a_misprint_and_the_correction():
    printed = np.array(_gold("paper_tensors.json")["Z_as_printed"]["re"])
    S = tensornet.superop_1q(gates.Z)
    assert not np.allclose(S, printed)
    np.testing.assert_array_equal(S, np.diag([1, -1, -1, 1]))
    # the corrected tensor acts as rho -> Z rho Z^dagger (plain matrix product)
    for s in range(3):
        rho = _rand_rho(s)
        np.testing.assert_allclose(S @ _vec(rho), _vec(gates.Z @ rho @ gates.Z.conj().T), atol=1e-15)


def test_printed_cnot_nonzeros():
    idx = _gold("paper_tensors.json")["CNOT_nonzeros"]["indices"]
    S = tensornet.superop_2q(gates.CNOT)
    expect = np.zeros((4, 4, 4, 4))
    for s in idx:
        expect[tuple(int(c) for c in s)] = 1.0
    np.testing.assert_array_equal(S, expect)


@pytest.mark.parametrize("name,P", [("M_Trace", gates.I2), ("M_X", gates.X), ("M_Y", gates.Y), ("M_Z", gates.Z)])
def test_printed_measurement_vectors(name, P):
    g = _gold("paper_tensors.json")[name]
    np.testing.assert_array_equal(tensornet.measure_vec(P), np.array(g["re"]) + 1j * np.array(g["im"]))


# --- superoperator identities (plain matrix algebra) ----------------------------------

def test_superop_1q_is_conjugation():
    for s in range(4):
        U = np.array(workloads.random_unitary(2, s))
        rho = _rand_rho(10 + s)
        np.testing.assert_allclose(tensornet.superop_1q(U) @ _vec(rho), _vec(U @ rho @ U.conj().T), atol=1e-14)


def test_superop_2q_is_conjugation():
    rng = np.random.default_rng(3)
    for s in range(3):
        U = np.array(workloads.random_unitary(4, s))
        a = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        rho = a @ a.conj().T
        out = U @ rho @ U.conj().T
        # rho on (q0, q1): rho[(a0 a1),(b0 b1)]; wire value of q_k is 2 a_k + b_k
        r4 = np.zeros((4, 4), dtype=complex)
        o4 = np.zeros((4, 4), dtype=complex)
        for a0, a1, b0, b1 in itertools.product(range(2), repeat=4):
            r4[2 * a0 + b0, 2 * a1 + b1] = rho[2 * a0 + a1, 2 * b0 + b1]
            o4[2 * a0 + b0, 2 * a1 + b1] = out[2 * a0 + a1, 2 * b0 + b1]
        got = np.tensordot(tensornet.superop_2q(U), r4, axes=([2, 3], [0, 1]))
        np.testing.assert_allclose(got, o4, atol=1e-13)


def test_measure_vec_gives_trace():
    for s in range(3):
        rho = _rand_rho(s)
        for P in (gates.I2, gates.X, gates.Y, gates.Z):
            assert abs(tensornet.measure_vec(P) @ _vec(rho) - np.trace(P @ rho)) < 1e-15


# --- state vector against textbook states ----------------------------------------------

def test_statevector_bell_and_rotation():
    psi = statevector.run(2, [("H", 0, -1, 0.0), ("CNOT", 0, 1, 0.0)])
    np.testing.assert_allclose(psi.ravel(), [2 ** -0.5, 0, 0, 2 ** -0.5], atol=1e-15)
    th = 0.7
    psi = statevector.run(1, [("RX", 0, -1, th)])
    np.testing.assert_allclose(np.abs(psi.ravel()) ** 2, [math.cos(th / 2) ** 2, math.sin(th / 2) ** 2], atol=1e-15)
    # qubit 0 is the most significant bit of the flat index
    psi = statevector.run(3, [("X", 0, -1, 0.0)])
    assert abs(psi.ravel()[4] - 1) < 1e-15


def test_zz_gate_is_diagonal_phase():
    th = 0.37
    d = np.diag(gates.zz(th))
    np.testing.assert_allclose(d, np.exp(-0.5j * th * np.array([1, -1, -1, 1])), atol=1e-15)
    assert np.count_nonzero(gates.zz(th) - np.diag(d)) == 0


# --- QAOA: known optimum, special cases, closed form vs state vector ------------------------

CUBE = [(0, 1), (0, 2), (0, 4), (1, 3), (1, 5), (2, 3), (2, 6), (3, 7), (4, 5), (4, 6), (5, 7), (6, 7)]


def test_triangle_free_3regular_optimum_statevector():
    """The 3-cube is 3-regular and triangle-free: each edge reaches 0.69245 at p=1."""
    g = _gold("qaoa_p1_known_values.json")["triangle_free_3regular_max_edge_cost"]
    gamma = 0.5 * math.asin(1 / math.sqrt(3))
    beta = math.pi / 8
    # sign: with exp(-i gamma ZZ) the cut-maximising branch has sin 2gamma sin 4beta < 0
    zz = statevector.qaoa_zz(8, CUBE, [-gamma], [beta])
    np.testing.assert_allclose((1 - zz) / 2, g["value"], atol=1e-14)
    zz_tn = tensornet.qaoa_zz(8, CUBE, [-gamma], [beta])
    np.testing.assert_allclose((1 - zz_tn) / 2, g["value"], atol=1e-13)
    np.testing.assert_allclose(closed_form.zz_p1(8, CUBE, -gamma, beta), zz, atol=1e-14)


@pytest.mark.parametrize("gamma,beta", [(0.0, 0.3), (0.4, 0.0)])
def test_zero_angle_cases(gamma, beta):
    e = workloads.random_regular_graph(3, 10, 1)
    zz = statevector.qaoa_zz(10, e, [gamma], [beta])
    np.testing.assert_allclose(zz, 0.0, atol=1e-14)
    np.testing.assert_allclose(tensornet.qaoa_zz(10, e, [gamma], [beta]), 0.0, atol=1e-14)
    np.testing.assert_allclose(closed_form.zz_p1(10, e, gamma, beta), 0.0, atol=1e-15)


@pytest.mark.parametrize("d,n,seed", [(3, 12, 0), (3, 12, 1), (3, 10, 5), (4, 10, 0), (5, 12, 2)])
def test_closed_form_matches_statevector(d, n, seed):
    e = workloads.random_regular_graph(d, n, seed)
    for gamma, beta in workloads.qaoa_angles(seed, 3, 1):
        np.testing.assert_allclose(closed_form.zz_p1(n, e, gamma, beta), statevector.qaoa_zz(n, e, [gamma], [beta]), atol=1e-13)


def test_graphs_with_triangles_are_covered():
    # the pins above must exercise the triangle term: count triangles of those graphs
    tri = 0
    for d, n, seed in [(3, 12, 0), (4, 10, 0), (5, 12, 2)]:
        e = workloads.random_regular_graph(d, n, seed)
        nb = [set() for _ in range(n)]
        for u, v in e:
            nb[u].add(v)
            nb[v].add(u)
        tri += sum(len(nb[u] & nb[v]) for u, v in e)
    assert tri > 0


def test_config1_reference_value():
    """The 12-vertex 3-regular p=1 instance at gamma=0.4, beta=0.3 (state vector)."""
    e = workloads.random_regular_graph(3, 12, 0)
    c_sv = statevector.qaoa_cost(12, e, [0.4], [0.3])
    assert abs(c_sv - closed_form.cost_p1(12, e, 0.4, 0.3)) < 1e-12
    assert 0 <= c_sv <= len(e)


# --- tensor network against the state vector ---------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_tn_expectation_matches_statevector(seed):
    n = 4
    gl = workloads.random_circuit(n, 10, seed)
    psi = statevector.run(n, gl)
    rng = workloads.SplitMix64(seed)
    for _ in range(3):
        pauli = [rng.below(4) for _ in range(n)]
        ref = statevector.expect_pauli(psi, pauli)
        got = tensornet.expectation(n, gl, pauli)
        assert abs(got - ref) < 1e-13
        got_lc = tensornet.expectation(n, gl, pauli, lightcone=True)
        assert abs(got_lc - ref) < 1e-13
        dbl = tensornet.contract(tensornet.doubled_network(n, gl, [gates.PAULI[c] for c in pauli]))
        assert abs(dbl - ref) < 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_tn_amplitude_and_probability(seed):
    n = 4
    gl = workloads.random_circuit(n, 12, 100 + seed)
    init = [np.array(workloads.random_unitary(2, 50 + q))[:, 0] for q in range(n)]
    psi = statevector.run(n, gl, statevector.product_state(init))
    total = 0.0
    for bits in itertools.product(range(2), repeat=n):
        amp = tensornet.amplitude(n, gl, bits, init)
        assert abs(amp - psi[bits]) < 1e-13
        pr = tensornet.probability(n, gl, bits, init)
        assert abs(pr - abs(psi[bits]) ** 2) < 1e-13
        total += pr.real
    assert abs(total - 1) < 1e-13
    # marginal: qubit 0 measured, others traced
    for b in range(2):
        m = tensornet.probability(n, gl, [b, 2, 2, 2], init)
        assert abs(m - np.sum(np.abs(psi[b]) ** 2)) < 1e-13


def test_all_trace_network_is_one():
    gl = workloads.random_circuit(5, 20, 7)
    assert abs(tensornet.expectation(5, gl, [0] * 5) - 1) < 1e-13


def test_tn_order_independence():
    n = 4
    gl = workloads.random_circuit(n, 10, 3)
    net = tensornet.folded_network(n, gl, [gates.Z, gates.I2, gates.X, gates.Z])
    wires = sorted({w for legs in net.legs for w in legs})
    vals = []
    for s in range(4):
        order = list(wires)
        np.random.default_rng(s).shuffle(order)
        vals.append(tensornet.contract(net, order))
    assert max(abs(v - vals[0]) for v in vals) < 1e-13


def test_tn_qaoa_matches_statevector_p2():
    e = workloads.random_regular_graph(3, 10, 2)
    ang = workloads.qaoa_angles(2, 1, 2)[0]
    ref = statevector.qaoa_zz(10, e, ang[:2], ang[2:])
    got = tensornet.qaoa_zz(10, e, ang[:2], ang[2:])
    np.testing.assert_allclose(got, ref, atol=1e-13)


# --- gradients ---------------------------------------------------------------------------

def test_parameter_shift_matches_closed_form_derivative():
    e = workloads.random_regular_graph(3, 10, 4)
    for gamma, beta in workloads.qaoa_angles(4, 2, 1):
        dg, db = closed_form.zz_p1_grad(10, e, gamma, beta)
        ps = gradients.parameter_shift(10, e, [gamma, beta])
        np.testing.assert_allclose(ps, [-0.5 * dg.sum(), -0.5 * db.sum()], atol=1e-11)


def test_closed_form_derivative_matches_fd_of_closed_form():
    e = workloads.random_regular_graph(4, 10, 1)
    g, b, h = 0.31, 0.77, 1e-6
    dg, db = closed_form.zz_p1_grad(10, e, g, b)
    fdg = (closed_form.zz_p1(10, e, g + h, b) - closed_form.zz_p1(10, e, g - h, b)) / (2 * h)
    fdb = (closed_form.zz_p1(10, e, g, b + h) - closed_form.zz_p1(10, e, g, b - h)) / (2 * h)
    np.testing.assert_allclose(dg, fdg, atol=1e-8)
    np.testing.assert_allclose(db, fdb, atol=1e-8)


def test_finite_difference_vs_parameter_shift_p2():
    e = workloads.random_regular_graph(3, 8, 6)
    params = workloads.qaoa_angles(6, 1, 2)[0]
    fd = gradients.finite_difference(8, e, params)
    ps = gradients.parameter_shift(8, e, params)
    np.testing.assert_allclose(fd, ps, atol=1e-5 * max(1, np.abs(ps).max()))


# --- light-cone state vectors (the route for graphs too large for a full state vector) ----------

@pytest.mark.parametrize("d,n,p,seed", [(3, 12, 1, 0), (3, 10, 2, 1), (4, 10, 2, 3)])
def test_lightcone_statevector_matches_full(d, n, p, seed):
    e = workloads.random_regular_graph(d, n, seed)
    ang = workloads.qaoa_angles(seed, 1, p)[0]
    full = statevector.qaoa_zz(n, e, ang[:p], ang[p:])
    lc = np.array([statevector.qaoa_zz_edge(n, e, ang[:p], ang[p:], ed) for ed in e])
    np.testing.assert_allclose(lc, full, atol=1e-13)
    m, _, _ = statevector.qaoa_edge_lightcone_circuit(n, e, ang[:p], ang[p:], e[0])
    assert m <= n


def test_edge_parameter_shift_sums_to_full_gradient():
    e = workloads.random_regular_graph(3, 8, 6)
    params = workloads.qaoa_angles(6, 1, 2)[0]
    full = gradients.parameter_shift(8, e, params)
    per_edge = sum(-0.5 * gradients.parameter_shift_edge(8, e, params, ed) for ed in e)
    np.testing.assert_allclose(per_edge, full, atol=1e-12)


def test_tn_parameter_shift_sums_to_full_gradient():
    """The light-cone tensor-network shift rule (used for the wide p=2 cones of
    the batching configuration) summed over all edges equals the full-state
    parameter shift, and each edge's entries equal the light-cone state-vector
    shift rule."""
    e = workloads.random_regular_graph(4, 8, 2)
    params = workloads.qaoa_angles(8, 1, 2)[0]
    full = gradients.parameter_shift(8, e, params)
    per = [gradients.parameter_shift_edge_tn(8, e, np.array(params), ed) for ed in e]
    np.testing.assert_allclose(sum(-0.5 * g for g in per), full, atol=1e-12)
    for ed, g in zip(e[:3], per):
        np.testing.assert_allclose(g, gradients.parameter_shift_edge(8, e, params, ed), atol=1e-12)


def test_config3_golden_values_are_consistent():
    """tests/golden/config3_p2.json (written by make_config3_p2.py from the
    oracle): one stored value recomputed, every <Z_u Z_v> in [-1, 1], and the
    stored gradient of one pair against central differences of the oracle's
    light-cone contraction (h = 1e-4; O(h^2) truncation)."""
    import json
    import os
    from oracle import gates as og
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config3_p2.json")))
    g = next(x for x in gold["graphs"] if (x["d"], x["n"]) == (4, 50))
    e = workloads.random_regular_graph(4, 50, 0)
    ang = np.array(workloads.qaoa_angles(0, 64, 2))
    for gg in gold["graphs"]:
        assert all(-1.0 <= v <= 1.0 for _, _, v in gg["values"])

    def zz(prm, edge):
        gl = og.qaoa_gate_list(50, e, prm[:2], prm[2:])[50:]
        pauli = [0] * 50
        pauli[edge[0]] = pauli[edge[1]] = 3
        return tensornet.expectation(50, gl, pauli, init=[np.array([1.0, 1.0]) / np.sqrt(2.0)] * 50,
                                     lightcone=True).real

    i, s, v = g["values"][0]
    assert abs(zz(ang[s], e[i]) - v) < 1e-13
    i, s, gv = g["grads"][0]
    h = 1e-4
    fd = []
    for k in range(4):
        d = np.zeros(4)
        d[k] = h
        fd.append((zz(ang[s] + d, e[i]) - zz(ang[s] - d, e[i])) / (2 * h))
    np.testing.assert_allclose(gv, fd, atol=1e-6)
