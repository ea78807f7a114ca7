"""GPU checks of the rows built past the hot path: the angle-optimisation
loop on the adjoint gradient, answer-string estimation and noise channels,
each against the FP64 oracle (complex64 tolerances as in test_gpu_parity)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads
from oracle import gradients

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CUBE = [(0, 1), (0, 2), (0, 4), (1, 3), (1, 5), (2, 3), (2, 6), (3, 7), (4, 5), (4, 6), (5, 7), (6, 7)]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03636_amd import qtn
    qtn.lib()


def _mods():
    from paper_1709_03636_amd import optimize, qaoa, qtn
    return optimize, qaoa, qtn


# --- angle optimisation (Adam on tn_batch_grad) ------------------------------------------

def test_angle_optimisation_reaches_p1_optimum_on_the_3cube():
    optimize, qaoa, qtn = _mods()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "qaoa_p1_known_values.json")))
    best = len(CUBE) * gold["triangle_free_3regular_max_edge_cost"]["value"]
    _say("optimise p=1 3-cube, 8 starts")
    model = qaoa.MaxCut(8, CUBE, 1, qtn.TN_C64, max_sets=8)
    xb, fb, trace = optimize.maxcut_optimize(model, workloads.qaoa_angles(3, 8, 1), steps=400, lr=0.05)
    torch.cuda.synchronize()
    fmax = float(fb.max())
    assert fmax <= best * (1 + 1e-5) and fmax >= best * (1 - 1e-5)
    x = xb[int(fb.argmax())].cpu().tolist()
    assert abs(gradients.cost(8, CUBE, x) - fmax) <= 1e-5 * best
    assert float(trace[-1]) >= float(trace[0])


def test_angle_optimisation_p2_beats_p1():
    optimize, qaoa, qtn = _mods()
    n = 10
    e = workloads.random_regular_graph(3, n, 4)
    res = {}
    for p in (1, 2):
        _say(f"optimise p={p} n={n}")
        model = qaoa.MaxCut(n, e, p, qtn.TN_C64, max_sets=8)
        xb, fb, _ = optimize.maxcut_optimize(model, workloads.qaoa_angles(7, 8, p), steps=300, lr=0.05)
        torch.cuda.synchronize()
        k = int(fb.argmax())
        res[p] = (float(fb[k]), xb[k].cpu().tolist())
        ref = gradients.cost(n, e, res[p][1])
        assert abs(ref - res[p][0]) <= 1e-5 * max(1.0, abs(ref))
    assert res[2][0] >= res[1][0] - 1e-5


# --- answer-string estimation (Sec. "Estimating the answer string") -------------------------

def test_answer_string_random_circuit_matches_oracle():
    from helpers import random_param_circuit
    from oracle import answer as oracle_answer, statevector
    _, _, qtn = _mods()
    from paper_1709_03636_amd import answer
    n = 7
    prod, ogates, params = random_param_circuit(n, 30, 21)
    draws = [k % 2 for k in range(n)]
    _say("answer string random circuit n=7 c128")
    bits, probs = answer.answer_string(n, prod, n_params=3, params=params, dtype=qtn.TN_C128, tie_tol=1e-9,
                                       tie_draws=draws)
    psi = statevector.run(n, ogates(params))
    rbits, rprobs = oracle_answer.answer_string(psi, 1e-9, draws)
    assert bits == rbits
    np.testing.assert_allclose(np.array(probs), np.array(rprobs), atol=1e-12)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_answer_string_qaoa_matches_oracle(dtype):
    from oracle import answer as oracle_answer, statevector
    _, qaoa, qtn = _mods()
    from paper_1709_03636_amd import answer
    n = 12
    e = workloads.random_regular_graph(3, n, 0)
    gam, bet = -0.35, 0.42
    gates_ = qaoa.qaoa_gates(n, e, 1)
    init = np.array([complex(qaoa.PLUS[0], qaoa.PLUS[1]), complex(qaoa.PLUS[2], qaoa.PLUS[3])] * n)
    draws = [1] + [0] * (n - 1)
    dt, tol, ptol = (qtn.TN_C128, 1e-9, 1e-12) if dtype == "c128" else (qtn.TN_C64, 1e-4, 1e-6)
    _say(f"answer string QAOA n={n} {dtype}")
    bits, probs = answer.answer_string(n, gates_, init=init, n_params=2, params=[gam, bet], dtype=dt, tie_tol=tol,
                                       tie_draws=draws)
    psi = statevector.qaoa_state(n, e, [gam], [bet])
    rbits, rprobs = oracle_answer.answer_string(psi, tol, draws)
    # the cost is symmetric under flipping every bit: qubit 0 is an exact tie and takes the draw
    assert abs(probs[0][0] - probs[0][1]) <= ptol and bits[0] == 1
    assert bits == rbits
    np.testing.assert_allclose(np.array(probs), np.array(rprobs), atol=ptol)
    assert answer.cut_value(e, bits) == sum(1 for u, v in e if rbits[u] != rbits[v])


# --- noise channels as superoperators -----------------------------------------------------

def _noisy_circuit(n, seed, non_tp=False):
    """(product gates, oracle ops factory, params): a seeded circuit with
    channels after some gates: depolarizing, amplitude damping, dephasing,
    and a two-qubit channel from a random isometry (all trace preserving),
    optionally one projection (not trace preserving)."""
    from helpers import random_param_circuit
    from oracle import gates as ogates_mod
    from paper_1709_03636_amd import noise
    prod, ogates, params = random_param_circuit(n, 18, seed)
    rng = np.random.default_rng(seed + 1000)
    chans = []  # (position after gate i, kraus, qubits)
    for i in range(len(prod)):
        r = rng.integers(0, 6)
        q = int(rng.integers(0, n))
        if r == 0:
            chans.append((i, noise.depolarizing(float(rng.uniform(0, 0.3))), [q]))
        elif r == 1:
            chans.append((i, noise.amplitude_damping(float(rng.uniform(0, 0.5))), [q]))
        elif r == 2:
            chans.append((i, noise.dephasing(float(rng.uniform(0, 0.4))), [q]))
        elif r == 3:
            q1 = (q + 1 + int(rng.integers(0, n - 1))) % n
            z = rng.normal(size=(16, 4)) + 1j * rng.normal(size=(16, 4))
            V, _ = np.linalg.qr(z)
            chans.append((i, [_kraus_of(V, k) for k in range(4)], [q, q1]))
    if non_tp:
        chans.append((len(prod) // 2, [np.diag([0.0, 1.0])], [1]))
    prod_n, layout = [], []
    for i, g in enumerate(prod):
        prod_n.append(g)
        layout.append(("g", i))
        for pos, kraus, qs in chans:
            if pos == i:
                prod_n.append(noise.channel_gate(kraus, qs[0], qs[1] if len(qs) > 1 else -1))
                layout.append(("c", kraus, qs))

    def oracle_ops(prm):
        og = ogates(prm)
        ops = []
        for item in layout:
            if item[0] == "g":
                k, q0, q1, th, ms = og[item[1]]
                ops.append(([ogates_mod.gate_matrix(k, th, ms)], [q0] if q1 < 0 else [q0, q1]))
            else:
                ops.append((item[1], item[2]))
        return ops

    return prod_n, oracle_ops, params


def _kraus_of(V, k):
    # rows 4k..4k+3 of a 16 x 4 isometry: four 4 x 4 Kraus operators with sum E^dagger E = I
    return V[4 * k:4 * k + 4, :]


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noisy_circuits_match_density_oracle(seed, dtype):
    from oracle import density, statevector
    _, _, qtn = _mods()
    n = 5
    prod, oracle_ops, params = _noisy_circuit(n, seed)
    rho = density.run(n, oracle_ops(params), density.pure(statevector.zero_state(n)))
    dt, tol = (qtn.TN_C128, 1e-12) if dtype == "c128" else (qtn.TN_C64, 1e-5)
    rng = np.random.default_rng(seed + 5)
    for case in range(4):
        pauli = [int(x) for x in rng.integers(0, 4, size=n)]
        bits = [int(x) for x in rng.integers(0, 3, size=n)]
        for mode, target, ref in ((qtn.TN_EXPECTATION, pauli, density.expect_pauli(rho, pauli)),
                                  (qtn.TN_PROBABILITY, bits, density.probability(rho, bits))):
            vals = []
            for lc in (True, False):
                _say(f"noisy seed={seed} {dtype} case={case} mode={mode} lightcone={lc}")
                net = qtn.Network(n, prod, mode, target, n_params=3, dtype=dt, lightcone=lc)
                net.set_order(net.order_linegraph(trials=4, seed=0))
                vals.append(net.contract(params))
            for v in vals:
                assert abs(v - ref) <= tol, (mode, target, v, ref)


def test_noisy_gradient_matches_finite_differences():
    from oracle import density, statevector
    _, _, qtn = _mods()
    n = 4
    prod, oracle_ops, params = _noisy_circuit(n, 3)
    pauli = [3, 1, 0, 3]
    net = qtn.Network(n, prod, qtn.TN_EXPECTATION, pauli, n_params=3, dtype=qtn.TN_C128)
    net.set_order(net.order_linegraph(trials=4, seed=0))
    _say("noisy gradient c128")
    val, g = net.grad(params)

    def f(prm):
        rho = density.run(n, oracle_ops(prm), density.pure(statevector.zero_state(n)))
        return density.expect_pauli(rho, pauli).real

    h = 1e-5
    fd = np.array([(f(params + h * np.eye(3)[i]) - f(params - h * np.eye(3)[i])) / (2 * h) for i in range(3)])
    assert abs(val - f(params)) < 1e-12
    np.testing.assert_allclose(g, fd, atol=1e-8)


def test_non_trace_preserving_map_turns_the_light_cone_off():
    from oracle import density, statevector
    _, _, qtn = _mods()
    n = 5
    prod, oracle_ops, params = _noisy_circuit(n, 4, non_tp=True)
    rho = density.run(n, oracle_ops(params), density.pure(statevector.zero_state(n)))
    bits = [0, 2, 2, 2, 2]
    on = qtn.Network(n, prod, qtn.TN_PROBABILITY, bits, n_params=3, dtype=qtn.TN_C128, lightcone=True)
    off = qtn.Network(n, prod, qtn.TN_PROBABILITY, bits, n_params=3, dtype=qtn.TN_C128, lightcone=False)
    assert on.wires()[1] == off.wires()[1]
    on.set_order(on.order_linegraph(trials=4, seed=0))
    _say("non-trace-preserving map")
    v = on.contract(params)
    assert abs(v - density.probability(rho, bits)) < 1e-12
    assert abs(density.probability(rho, [2] * n).real - 1.0) > 1e-3  # the projection removed weight


def test_noisy_qaoa_maxcut_matches_density_oracle():
    from oracle import density, gates as og, statevector
    from paper_1709_03636_amd import noise
    _, qaoa, qtn = _mods()
    n = 8
    e = workloads.random_regular_graph(3, n, 2)
    K = noise.depolarizing(0.05)
    S = 3
    ang = workloads.qaoa_angles(6, S, 1)
    _say("noisy QAOA MaxCut n=8")
    model = qaoa.MaxCut(n, e, 1, qtn.TN_C128, order="linegraph", max_sets=S, noise=K)
    obj, grad = model.value_and_grad(torch.tensor(ang, dtype=torch.float64, device="cuda"))
    obj = obj.cpu().numpy()
    for s in range(S):
        gam, bet = ang[s]
        ops = [([og.gate_matrix("H")], [q]) for q in range(n)]
        for u, v in e:
            ops += [([og.zz(2 * gam)], [u, v]), (K, [u]), (K, [v])]
        for q in range(n):
            ops += [([og.rot(og.X, 2 * bet)], [q]), (K, [q])]
        rho = density.run(n, ops, density.pure(statevector.zero_state(n)))
        ref = sum((1 - density.expect_pauli(rho, [3 if q in (u, v) else 0 for q in range(n)]).real) / 2
                  for u, v in e)
        assert abs(obj[s] - ref) < 1e-10 * len(e)


# --- diagonal gates as hyperedge tensors (tn_target.diagonal) --------------------------------

def _diag_circuit(n, seed):
    """Seeded circuit (RZ, ZZ, CZ, Z among the generic gates) plus explicit
    diagonal one- and two-qubit custom gates; returns (product gates, oracle
    apply(params) -> state, params)."""
    from helpers import random_param_circuit
    from oracle import gates as og, statevector
    prod, ogates, params = random_param_circuit(n, 36, seed)
    rng = np.random.default_rng(seed + 300)
    extra = []
    for _ in range(4):
        q = int(rng.integers(0, n))
        extra.append(("U1", q, -1, np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 2)))))
        q0, q1 = rng.choice(n, 2, replace=False)
        extra.append(("U2", int(q0), int(q1), np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 4)))))
    # interleave: one extra gate after every 4 generic gates
    prod_all, order = [], []
    for i, g in enumerate(prod):
        prod_all.append(g)
        order.append(("g", i))
        if i % 4 == 3 and i // 4 < len(extra):
            k, q0, q1, M = extra[i // 4]
            prod_all.append((k, q0, q1, -1, 0.0, M))
            order.append(("x", i // 4))

    def state(prm):
        gl = ogates(prm)
        psi = statevector.zero_state(n)
        for kind, idx in order:
            if kind == "g":
                k, q0, q1, th, ms = gl[idx]
                U = og.gate_matrix(k, th, ms)
            else:
                k, q0, q1, U = extra[idx]
            psi = statevector.apply_1q(psi, U, q0) if q1 < 0 else statevector.apply_2q(psi, U, q0, q1)
        return psi

    return prod_all, state, params


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_diagonal_mode_random_circuits_all_modes(seed):
    from oracle import statevector
    _, _, qtn = _mods()
    n = 6
    prod, state, params = _diag_circuit(n, seed)
    psi = state(params)
    rng = np.random.default_rng(seed + 7)
    pauli = [int(x) for x in rng.integers(0, 4, size=n)]
    bits_p = [int(x) for x in rng.integers(0, 3, size=n)]
    bits_a = [int(x) for x in rng.integers(0, 2, size=n)]
    prob = np.abs(psi) ** 2
    for q in reversed(range(n)):
        prob = prob.sum(axis=q) if bits_p[q] == 2 else np.take(prob, bits_p[q], axis=q)
    cases = ((qtn.TN_EXPECTATION, pauli, statevector.expect_pauli(psi, pauli)),
             (qtn.TN_PROBABILITY, bits_p, float(prob)),
             (qtn.TN_AMPLITUDE, bits_a, psi[tuple(bits_a)]))
    for mode, target, ref in cases:
        dense = qtn.Network(n, prod, mode, target, n_params=3, dtype=qtn.TN_C128)
        diag = qtn.Network(n, prod, mode, target, n_params=3, dtype=qtn.TN_C128, diagonal=True)
        assert diag.wires()[0] < dense.wires()[0]  # diagonal gates add no wires
        for net in (diag,):
            for pi in (net.order_stochastic(seed), net.order_linegraph(trials=4, seed=seed)):
                _say(f"diagonal seed={seed} mode={mode}")
                net.set_order(pi)
                v = net.contract(params)
                assert abs(v - ref) <= 1e-12 * max(1.0, abs(ref)), (mode, v, ref)


def test_diagonal_mode_gradient_matches_finite_differences():
    from oracle import statevector
    _, _, qtn = _mods()
    n = 6
    prod, state, params = _diag_circuit(n, 5)
    pauli = [3, 0, 1, 3, 2, 0]
    net = qtn.Network(n, prod, qtn.TN_EXPECTATION, pauli, n_params=3, dtype=qtn.TN_C128, diagonal=True)
    net.set_order(net.order_linegraph(trials=4, seed=0))
    _say("diagonal gradient c128")
    val, g = net.grad(params)

    def f(prm):
        return statevector.expect_pauli(state(prm), pauli).real

    h = 1e-5
    fd = np.array([(f(params + h * np.eye(3)[i]) - f(params - h * np.eye(3)[i])) / (2 * h) for i in range(3)])
    assert abs(val - f(params)) < 1e-12
    np.testing.assert_allclose(g, fd, atol=1e-8)


@pytest.mark.parametrize("cfg", ["records", "sets", "block128", "block256", "global", "level"])
def test_diagonal_qaoa_batch_every_executor(cfg, monkeypatch):
    """Hyperedge (batch-label) steps through every executor: 64-lane lane
    records, set-packed records, the descriptor path at 128/256 lanes, the
    global-arena fused executor and the level executor; p=1 values and
    gradients against the closed form."""
    from oracle import closed_form
    _, qaoa, qtn = _mods()
    env = {"records": {"QTN_SETS_PER_WAVE": "1", "QTN_FUSED_BLOCK": "64"},
           "sets": {"QTN_SETS_PER_WAVE": "4", "QTN_FUSED_BLOCK": "64"},
           "block128": {"QTN_SETS_PER_WAVE": "1", "QTN_FUSED_BLOCK": "128"},
           "block256": {"QTN_SETS_PER_WAVE": "1", "QTN_FUSED_BLOCK": "256"},
           "global": {"QTN_FUSED_LDS_MAX": "0"},
           "level": {"QTN_FUSED_LDS_MAX": "0", "QTN_GMEM_MAX_MACS": "0"}}[cfg]
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    n, d = 20, 3
    e = workloads.random_regular_graph(d, n, 3)
    S = 6
    ang = workloads.qaoa_angles(4, S, 1)
    for dt, tol, gtol in ((qtn.TN_C128, 1e-12, 1e-10), (qtn.TN_C64, 1e-5, 1e-4)):
        _say(f"diagonal QAOA batch {cfg} dtype={dt}")
        model = qaoa.MaxCut(n, e, 1, dt, order="linegraph", max_sets=S, diagonal=True)
        info = model.batch.info()
        if cfg == "level":
            assert info["n_level"] == len(e)
        if cfg == "global":
            assert info["n_global"] == len(e)
        out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
        obj, grad = model.value_and_grad(torch.tensor(ang, dtype=torch.float64, device="cuda"), out=out)
        torch.cuda.synchronize()
        o, grad = out.cpu().numpy(), grad.cpu().numpy()
        for s in range(S):
            zz = closed_form.zz_p1(n, e, ang[s][0], ang[s][1])
            assert np.max(np.abs(o[:, s, 0] - zz)) < tol
            dg, db = closed_form.zz_p1_grad(n, e, ang[s][0], ang[s][1])
            g_ref = np.array([-0.5 * dg.sum(), -0.5 * db.sum()])
            assert np.max(np.abs(grad[s] - g_ref)) <= gtol * max(1, np.abs(g_ref).max())


def test_diagonal_qaoa_p2_matches_statevector():
    _, qaoa, qtn = _mods()
    n = 12
    e = workloads.random_regular_graph(3, n, 6)
    S = 3
    ang = workloads.qaoa_angles(8, S, 2)
    _say("diagonal QAOA p=2")
    model = qaoa.MaxCut(n, e, 2, qtn.TN_C128, order="stochastic", max_sets=S, diagonal=True)
    obj, grad = model.value_and_grad(torch.tensor(ang, dtype=torch.float64, device="cuda"))
    obj, grad = obj.cpu().numpy(), grad.cpu().numpy()
    for s in range(S):
        ref = gradients.cost(n, e, list(ang[s]))
        ps = gradients.parameter_shift(n, e, list(ang[s]))
        assert abs(obj[s] - ref) < 1e-11
        np.testing.assert_allclose(grad[s], ps, atol=1e-10)


def test_diagonal_mode_with_noise():
    from oracle import density, gates as og, statevector
    from paper_1709_03636_amd import noise
    _, qaoa, qtn = _mods()
    n = 8
    e = workloads.random_regular_graph(3, n, 2)
    K = noise.amplitude_damping(0.07)
    ang = workloads.qaoa_angles(9, 2, 1)
    _say("diagonal + noise")
    model = qaoa.MaxCut(n, e, 1, qtn.TN_C128, order="linegraph", max_sets=2, noise=K, diagonal=True)
    obj = model.expectation(torch.tensor(ang, dtype=torch.float64, device="cuda")).cpu().numpy()
    for s in range(2):
        gam, bet = ang[s]
        ops = [([og.gate_matrix("H")], [q]) for q in range(n)]
        for u, v in e:
            ops += [([og.zz(2 * gam)], [u, v]), (K, [u]), (K, [v])]
        for q in range(n):
            ops += [([og.rot(og.X, 2 * bet)], [q]), (K, [q])]
        rho = density.run(n, ops, density.pure(statevector.zero_state(n)))
        ref = sum((1 - density.expect_pauli(rho, [3 if q in (u, v) else 0 for q in range(n)]).real) / 2
                  for u, v in e)
        assert abs(obj[s] - ref) < 1e-10 * len(e)


def test_diagonal_whole_circuit_6regular_n30():
    """The dense regime's whole-circuit network of one edge (6-regular, n=30,
    p=1, trace on every other qubit): with dense gates its orders need
    intermediates of 2^42 entries or more; in diagonal mode the line-graph
    order peaks at 2^28. Its value against the p=1 closed form."""
    from oracle import closed_form
    _, qaoa, qtn = _mods()
    n = 30
    e = workloads.random_regular_graph(6, n, 0)
    net = qaoa.edge_network(n, e, 1, e[0], dtype=qtn.TN_C64, lightcone=False, diagonal=True)
    net.set_order(net.order_linegraph(trials=8, seed=0))
    assert net.plan_info()["peak_bits"] <= 28
    gam, bet = 0.31, -0.52
    _say("whole circuit 6-regular n=30 diagonal")
    v = net.contract([gam, bet])
    ref = closed_form.zz_p1(n, e, gam, bet)[0]
    assert abs(v.real - ref) < 1e-5 and abs(v.imag) < 1e-5


# --- degenerate cases ----------------------------------------------------------------------

def test_circuits_without_gates_and_single_qubits():
    """No gates at all (the network is the initial state against the
    measurement) and one-qubit circuits, in every mode and both orders."""
    _, _, qtn = _mods()
    rng = np.random.default_rng(11)
    for n in (1, 3):
        v = rng.normal(size=(n, 2)) + 1j * rng.normal(size=(n, 2))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        init = v.reshape(-1)
        for gates_ in ([], [("H", 0, -1, -1, 0.0), ("RY", 0, -1, 0, 0.7)]):
            psi = v[0]
            if gates_:
                from oracle import gates as og
                psi = og.rot(og.Y, 0.7 * 0.3) @ (og.H @ v[0])
            full = [psi] + [v[q] for q in range(1, n)]
            X = np.array([[0, 1], [1, 0]])
            Z = np.diag([1.0, -1.0])
            exp_ref = np.prod([np.vdot(full[q], (Z if q == 0 else X) @ full[q]) for q in range(n)])
            prob_ref = abs(full[0][1]) ** 2 * np.prod([abs(full[q][0]) ** 2 for q in range(1, n)])
            amp_ref = full[0][1] * np.prod([full[q][0] for q in range(1, n)])
            cases = ((qtn.TN_EXPECTATION, [3] + [1] * (n - 1), exp_ref), (qtn.TN_PROBABILITY, [1] + [0] * (n - 1), prob_ref),
                     (qtn.TN_AMPLITUDE, [1] + [0] * (n - 1), amp_ref))
            for mode, target, ref in cases:
                net = qtn.Network(n, gates_, mode, target, n_params=1, init=init, dtype=qtn.TN_C128)
                for pi in (net.order_stochastic(1), net.order_linegraph(trials=2, seed=1)):
                    net.set_order(pi)
                    _say(f"degenerate n={n} gates={len(gates_)} mode={mode}")
                    val = net.contract([0.3])
                    assert abs(val - ref) < 1e-12, (n, len(gates_), mode, val, ref)


def test_disconnected_components_in_a_batch_with_gradient():
    """Qubit pairs that never interact: the network falls apart into
    components whose scalars multiply; values and gradients in a batch
    against the state vector and parameter shift."""
    from oracle import statevector
    _, _, qtn = _mods()
    gates_ = [("H", 0, -1, -1, 0.0), ("ZZ", 0, 1, 0, 1.0), ("RX", 1, -1, 1, 1.0),
              ("H", 2, -1, -1, 0.0), ("ZZ", 2, 3, 1, 0.5), ("RY", 3, -1, 0, 1.0)]
    pauli = [3, 3, 1, 3]
    nets = []
    for diag in (False, True):
        net = qtn.Network(4, gates_, qtn.TN_EXPECTATION, pauli, n_params=2, dtype=qtn.TN_C128, diagonal=diag)
        net.set_order(net.order_linegraph(trials=2, seed=0))
        nets.append(net)
    assert nets[0].plan_info()["n_components"] == 2
    ang = np.array([[0.4, -0.7], [1.1, 0.2], [-0.3, 0.9]])
    batch = qtn.Batch(nets, coef=[1.0, 0.0], max_sets=3)
    out = torch.empty((2, 3, 2), dtype=torch.float64, device="cuda")
    gnet = torch.empty((2, 3, 2), dtype=torch.float64, device="cuda")
    _say("disconnected components batch")
    batch.grad(torch.tensor(ang, device="cuda"), out=out, grad_net=gnet)
    torch.cuda.synchronize()
    out, gnet = out.cpu().numpy(), gnet.cpu().numpy()

    def f(prm):
        gl = [("H", 0, -1, 0.0), ("ZZ", 0, 1, prm[0]), ("RX", 1, -1, prm[1]), ("H", 2, -1, 0.0),
              ("ZZ", 2, 3, 0.5 * prm[1]), ("RY", 3, -1, prm[0])]
        return statevector.expect_pauli(statevector.run(4, gl), pauli).real

    for s in range(3):
        ref = f(ang[s])
        h = 1e-5
        fd = [(f(ang[s] + h * np.eye(2)[i]) - f(ang[s] - h * np.eye(2)[i])) / (2 * h) for i in range(2)]
        for k in range(2):
            assert abs(out[k, s, 0] - ref) < 1e-12
            np.testing.assert_allclose(gnet[k, s], fd, atol=1e-8)


def test_batch_without_parameters_and_set_bounds():
    _, _, qtn = _mods()
    gates_ = [("H", 0, -1, -1, 0.0), ("CNOT", 0, 1, -1, 0.0)]
    net = qtn.Network(2, gates_, qtn.TN_EXPECTATION, [3, 3], n_params=0, dtype=qtn.TN_C64)
    net.set_order(net.order_stochastic(0))
    batch = qtn.Batch([net], coef=[2.0], offset=1.0, max_sets=2)
    params = torch.empty((2, 0), dtype=torch.float64, device="cuda")
    out = torch.empty((1, 2, 2), dtype=torch.float64, device="cuda")
    obj = torch.empty(2, dtype=torch.float64, device="cuda")
    batch.contract(params, out=out, obj=obj)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out[0, :, 0].cpu().numpy(), [1.0, 1.0], atol=1e-6)  # Bell state: <ZZ> = 1
    np.testing.assert_allclose(obj.cpu().numpy(), [3.0, 3.0], atol=1e-6)
    with pytest.raises(qtn.QtnError):
        batch.contract(torch.empty((3, 0), dtype=torch.float64, device="cuda"))  # more sets than max_sets
