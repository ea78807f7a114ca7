"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: complex128 path vs the oracle 1e-12 (values) and 1e-10
(gradients); complex64 path (FP32 contraction, FP64 final scalars and
gradient sums) 1e-5 absolute for <Z_u Z_v>, probabilities and amplitudes
(scaled by the largest magnitude), 1e-5 relative for <C>, and
1e-4 * max(1, |g|) for gradients.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import workloads
from helpers import random_param_circuit
from oracle import closed_form, gradients, statevector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_03636_amd import qtn
    qtn.lib()  # loud failure when the library is not built


def _qtn():
    from paper_1709_03636_amd import qtn
    return qtn


def _qaoa():
    from paper_1709_03636_amd import qaoa
    return qaoa


# --- the 12-vertex 3-regular p=1 instance at gamma=0.4, beta=0.3 --------------------

@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_config1_per_edge(dtype, tol):
    qtn, qaoa = _qtn(), _qaoa()
    dt = qtn.TN_C128 if dtype == "c128" else qtn.TN_C64
    e = workloads.random_regular_graph(3, 12, 0)
    ref = statevector.qaoa_zz(12, e, [0.4], [0.3])
    nets = qaoa.edge_networks(12, e, 1, dt, order="stochastic", seed=0)
    got = []
    for i, net in enumerate(nets):
        _say(f"config1 {dtype} edge {i} {e[i]}")
        z = net.contract([0.4, 0.3])
        got.append(z)
    got = np.array(got)
    assert np.max(np.abs(got.real - ref)) < tol
    assert np.max(np.abs(got.imag)) < tol
    c_gpu = float(np.sum((1 - got.real) / 2))
    c_ref = float(np.sum((1 - ref) / 2))
    assert abs(c_gpu - c_ref) <= tol * max(1.0, abs(c_ref))


# --- random circuits in all three modes ---------------------------------------------------

@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
@pytest.mark.parametrize("seed", range(4))
def test_random_circuit_expectation(dtype, tol, seed):
    qtn = _qtn()
    dt = qtn.TN_C128 if dtype == "c128" else qtn.TN_C64
    n = 5
    prod, og, prm = random_param_circuit(n, 18, seed)
    psi = statevector.run(n, og(prm))
    rng = workloads.SplitMix64(seed)
    for t in range(3):
        pauli = [rng.below(4) for _ in range(n)]
        if not any(pauli):
            pauli[0] = 3
        ref = statevector.expect_pauli(psi, pauli)
        for lc in (True, False):
            _say(f"expect {dtype} seed {seed} pauli {pauli} lc {lc}")
            net = qtn.Network(n, prod, qtn.TN_EXPECTATION, pauli, n_params=len(prm), dtype=dt, lightcone=lc)
            net.set_order(net.order_stochastic(seed + t))
            got = net.contract(prm)
            assert abs(got - ref) < tol, (got, ref)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
@pytest.mark.parametrize("seed", range(3))
def test_random_circuit_amplitude_probability(dtype, tol, seed):
    qtn = _qtn()
    dt = qtn.TN_C128 if dtype == "c128" else qtn.TN_C64
    n = 4
    prod, og, prm = random_param_circuit(n, 14, 100 + seed)
    init = [np.array(workloads.random_unitary(2, 50 + q))[:, 0] for q in range(n)]
    psi = statevector.run(n, og(prm), statevector.product_state(init))
    scale = np.abs(psi).max()
    for bits in itertools.product(range(2), repeat=n):
        _say(f"amp/prob {dtype} seed {seed} bits {bits}")
        na = qtn.Network(n, prod, qtn.TN_AMPLITUDE, bits, n_params=len(prm), init=np.concatenate(init), dtype=dt)
        na.set_order(na.order_linegraph(trials=2, seed=seed))
        a = na.contract(prm)
        assert abs(a - psi[bits]) < tol * max(1.0, scale), (a, psi[bits])
        npb = qtn.Network(n, prod, qtn.TN_PROBABILITY, bits, n_params=len(prm), init=np.concatenate(init), dtype=dt)
        npb.set_order(npb.order_stochastic(seed))
        pr = npb.contract(prm)
        assert abs(pr - abs(psi[bits]) ** 2) < tol
    # marginal of qubit 1 (others traced)
    for b in range(2):
        bits = [2, b, 2, 2]
        net = qtn.Network(n, prod, qtn.TN_PROBABILITY, bits, n_params=len(prm), init=np.concatenate(init), dtype=dt)
        net.set_order(net.order_stochastic(1))
        ref = float(np.sum(np.abs(psi[:, b]) ** 2))
        assert abs(net.contract(prm) - ref) < tol


# --- gradients ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_grad_p1_vs_parameter_shift(dtype):
    qtn, qaoa = _qtn(), _qaoa()
    dt = qtn.TN_C128 if dtype == "c128" else qtn.TN_C64
    e = workloads.random_regular_graph(3, 10, 4)
    params = [0.37, 0.81]
    ps = gradients.parameter_shift(10, e, params)
    c_ref = gradients.cost(10, e, params)
    nets = qaoa.edge_networks(10, e, 1, dt, order="linegraph")
    tot_v, tot_g = 0.0, np.zeros(2)
    for i, net in enumerate(nets):
        _say(f"grad p1 {dtype} edge {i}")
        v, g = net.grad(params)
        tot_v += (1 - v) / 2
        tot_g += -0.5 * g
    vt, gt = (1e-12, 1e-10) if dtype == "c128" else (1e-5, 1e-4)
    assert abs(tot_v - c_ref) <= vt * max(1, abs(c_ref))
    assert np.max(np.abs(tot_g - ps)) <= gt * max(1, np.abs(ps).max())


def test_grad_p2_vs_parameter_shift_c128():
    qtn, qaoa = _qtn(), _qaoa()
    e = workloads.random_regular_graph(3, 8, 6)
    params = workloads.qaoa_angles(6, 1, 2)[0]
    ps = gradients.parameter_shift(8, e, params)
    nets = qaoa.edge_networks(8, e, 2, qtn.TN_C128, order="stochastic", seed=3)
    tot_g = np.zeros(4)
    for i, net in enumerate(nets):
        _say(f"grad p2 c128 edge {i}")
        _, g = net.grad(params)
        tot_g += -0.5 * g
    assert np.max(np.abs(tot_g - ps)) <= 1e-10 * max(1, np.abs(ps).max())


# --- batched path --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_p1_closed_form(dtype):
    qtn, qaoa = _qtn(), _qaoa()
    dt = qtn.TN_C128 if dtype == "c128" else qtn.TN_C64
    n, d = 30, 4
    e = workloads.random_regular_graph(d, n, 2)
    S = 16
    ang = np.array(workloads.qaoa_angles(9, S, 1))
    _say(f"batch p1 {dtype} n={n} d={d} S={S}")
    model = qaoa.MaxCut(n, e, 1, dt, order="linegraph", max_sets=S)
    out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    obj, grad = model.value_and_grad(torch.tensor(ang, device="cuda"), out=out)
    torch.cuda.synchronize()
    out, obj, grad = out.cpu().numpy(), obj.cpu().numpy(), grad.cpu().numpy()
    tol = 1e-12 if dtype == "c128" else 1e-5
    for s in range(S):
        zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
        assert np.max(np.abs(out[:, s, 0] - zz)) < tol
        c_ref = float(np.sum((1 - zz) / 2))
        assert abs(obj[s] - c_ref) <= tol * max(1, c_ref)
        dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
        g_ref = np.array([-0.5 * dg.sum(), -0.5 * db.sum()])
        gt = 1e-10 if dtype == "c128" else 1e-4
        assert np.max(np.abs(grad[s] - g_ref)) <= gt * max(1, np.abs(g_ref).max())


def test_batch_forward_matches_grad_pass_and_graph_replay():
    qtn, qaoa = _qtn(), _qaoa()
    n = 16
    e = workloads.random_regular_graph(3, n, 5)
    S = 8
    ang = torch.tensor(workloads.qaoa_angles(5, S, 2), device="cuda", dtype=torch.float64)
    model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="stochastic", max_sets=S)
    _say("batch eager fwd / grad")
    obj_f = model.expectation(ang)
    obj_g, grad_g = model.value_and_grad(ang)
    torch.cuda.synchronize()
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    assert np.max(np.abs(obj_f.cpu().numpy() - ref)) <= 1e-5 * max(1, np.abs(ref).max())
    assert np.max(np.abs(obj_g.cpu().numpy() - ref)) <= 1e-5 * max(1, np.abs(ref).max())
    st = torch.cuda.Stream()
    obj = torch.empty(S, dtype=torch.float64, device="cuda")
    grad = torch.empty((S, 4), dtype=torch.float64, device="cuda")
    for rep in range(3):
        _say(f"graph replay {rep}")
        obj.zero_()
        grad.zero_()
        st.wait_stream(torch.cuda.current_stream())
        model.batch.run_graph(True, ang, obj=obj, grad=grad, stream=st)
        st.synchronize()
        torch.cuda.synchronize()
        assert np.max(np.abs(obj.cpu().numpy() - ref)) <= 1e-5 * max(1, np.abs(ref).max())
        assert np.max(np.abs(grad.cpu().numpy() - grad_g.cpu().numpy())) <= 1e-6
        _ = (ang * 2).sum().item()  # eager work between replays


def test_kernel_timing_hook(monkeypatch):
    """tn_batch_kernel_timing records one event pair per eager executor
    launch and none inside graph captures; the results are unchanged. A batch
    split over the three executors (level networks on the task executor)
    times each executor on its own stream."""
    qtn, qaoa = _qtn(), _qaoa()
    n = 12
    e = workloads.random_regular_graph(3, n, 3)
    S = 4
    ang = torch.tensor(workloads.qaoa_angles(3, S, 1), device="cuda", dtype=torch.float64)
    model = qaoa.MaxCut(n, e, 1, qtn.TN_C64, max_sets=S)
    obj0, grad0 = model.value_and_grad(ang)
    st = torch.cuda.Stream()
    model.batch.kernel_timing(True)
    for _ in range(3):
        model.batch.grad(ang, stream=st)
    model.batch.contract(ang, stream=st)
    obj = torch.empty(S, dtype=torch.float64, device="cuda")
    st.wait_stream(torch.cuda.current_stream())
    model.batch.run_graph(False, ang, obj=obj, stream=st)
    st.synchronize()
    n_timed, ms = model.batch.kernel_time()
    assert n_timed == 4 and 0.0 < ms < 1e3
    assert model.batch.kernel_time() == (0, 0.0)
    model.batch.kernel_timing(False)
    obj1, grad1 = model.value_and_grad(ang)
    torch.cuda.synchronize()
    assert np.array_equal(obj0.cpu().numpy(), obj1.cpu().numpy())
    assert np.array_equal(grad0.cpu().numpy(), grad1.cpu().numpy())
    # forward-only graph vs the adjoint pass's value: different kernels, c64 tolerance
    assert np.max(np.abs(obj.cpu().numpy() - obj0.cpu().numpy())) <= 1e-5 * max(1.0, float(obj0.abs().max()))
    # three executors
    n = 24
    e = workloads.random_regular_graph(3, n, 2)
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "32768")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", str(1 << 18))
    monkeypatch.setenv("QTN_TASK_MIN", "1")
    monkeypatch.setenv("QTN_GMEM_JOIN", "0")
    model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="linegraph", max_sets=S, trials=2)
    info = model.batch.info()
    assert info["n_fused"] > 0 and info["n_global"] > 0 and info["n_level_tasked"] == info["n_level_groups"] == 1
    ang = torch.tensor(workloads.qaoa_angles(4, S, 2), device="cuda", dtype=torch.float64)
    obj0, grad0 = model.value_and_grad(ang)
    model.batch.kernel_timing(True)
    for _ in range(3):
        model.batch.grad(ang, stream=st)
    model.batch.contract(ang, stream=st)
    st.synchronize()
    _say("kernel timing, three executors")
    for ex in (qtn.TN_EXEC_FUSED, qtn.TN_EXEC_LEVEL, qtn.TN_EXEC_GLOBAL):
        n_timed, ms = model.batch.kernel_time(ex)
        assert n_timed == 4 and 0.0 < ms < 1e3, (ex, n_timed, ms)
        assert model.batch.kernel_time(ex) == (0, 0.0)
    model.batch.kernel_timing(False)
    obj1, grad1 = model.value_and_grad(ang)
    torch.cuda.synchronize()
    assert np.array_equal(obj0.cpu().numpy(), obj1.cpu().numpy())
    assert np.array_equal(grad0.cpu().numpy(), grad1.cpu().numpy())


def test_bind_params_kernel():
    """Angle binding on its own: RX and ZZ superoperators vs their definitions."""
    qtn, qaoa = _qtn(), _qaoa()
    e = [(0, 1)]
    net = qaoa.edge_network(2, e, 1, e[0], dtype=qtn.TN_C128)
    per = net.bind_params(None, 0)
    S = 3
    ang = torch.tensor([[0.3, 0.7], [1.1, -0.4], [2.0, 0.25]], dtype=torch.float64, device="cuda")
    out = torch.zeros((S, per, 2), dtype=torch.float64, device="cuda")
    _say("bind params")
    net.bind_params(ang, S, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    from oracle import gates as og, tensornet as tn
    for s in range(S):
        g, b = ang[s].cpu().numpy()
        zz = tn.superop_2q(og.zz(2 * g)).ravel()
        rx = tn.superop_1q(og.rot(og.X, 2 * b)).ravel()
        np.testing.assert_allclose(got[s][:256], zz, atol=1e-14)
        np.testing.assert_allclose(got[s][256:], rx, atol=1e-14)


def _mixed_level_budget(qtn, qaoa, n, e, S, monkeypatch):
    """A level-arena budget (bytes) under which the level networks split into
    several groups and, where the sizes allow, some run alone in chunks."""
    best = None
    for k in range(30, 8, -1):
        monkeypatch.setenv("QTN_LEVEL_BUDGET", str(1 << k))
        info = qaoa.MaxCut(n, e, 2, qtn.TN_C128, order="linegraph", max_sets=S).batch.info()
        if info["n_level_groups"] >= 2 and best is None:  # packed groups
            best = 1 << k
        if info["n_level_groups"] >= 2 and info["n_level_chunked"] >= 1:
            return 1 << k
    return best


@pytest.mark.parametrize("mode", ["item", "task"])
def test_level_group_many_items(mode, monkeypatch):
    """A large level group: 150 light-cone networks of a 3-regular n=100
    graph, p=1, all on the level executor in one group, run one launch per
    item (item mode) or by the task executor (450 tasks), against the p=1
    closed form and its derivative on every edge and parameter vector."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    monkeypatch.setenv("QTN_TASK_MIN", "1" if mode == "task" else "1000000000")
    n, S = 100, 3
    e = workloads.random_regular_graph(3, n, 0)
    ang = np.array(workloads.qaoa_angles(9, S, 1))
    nets = qaoa.edge_networks(n, e, 1, qtn.TN_C64, order="linegraph", trials=2)
    batch = qtn.Batch(nets, max_sets=S)
    info = batch.info()
    assert info["n_level"] == len(e) and info["n_level_groups"] == 1 and info["n_level_chunked"] == 0
    assert info["n_level_tasked"] == (mode == "task")
    out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    gn = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    _say(f"level group of {len(e)} networks, launches {info['level_launches_grad']}")
    batch.grad(torch.tensor(ang, device="cuda"), out=out, grad_net=gn)
    torch.cuda.synchronize()
    got, g = out.cpu().numpy(), gn.cpu().numpy()
    for s in range(S):
        zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
        dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
        assert np.max(np.abs(got[:, s, 0] - zz)) < 1e-5
        assert np.max(np.abs(g[:, s, 0] - dg)) < 1e-4 and np.max(np.abs(g[:, s, 1] - db)) < 1e-4


def test_level_executor_matches_fused(monkeypatch):
    """The same batch on the LDS fused executor, on the global-arena fused
    executor and on the level executor: all networks in one group, stepped
    together one launch per step (item mode) or run by the task executor, in
    several groups with some networks run alone (arena budget lowered), and
    every network alone in chunks of one parameter vector."""
    qtn, qaoa = _qtn(), _qaoa()
    n = 14
    e = workloads.random_regular_graph(3, n, 8)
    S = 5
    ang = torch.tensor(workloads.qaoa_angles(8, S, 2), device="cuda", dtype=torch.float64)
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    ps = np.array([gradients.parameter_shift(n, e, list(a)) for a in ang.cpu().numpy()])
    res = {}
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    mixed = _mixed_level_budget(qtn, qaoa, n, e, S, monkeypatch)
    assert mixed is not None
    for mode, lim, gmem, budget, tmin in (("fused", str(160 * 1024), None, None, None),
                                          ("global", "0", None, None, None), ("level", "0", "0", None, None),
                                          ("level-task", "0", "0", None, "1"),
                                          ("level-mixed", "0", "0", str(mixed), None),
                                          ("level-mixed-task", "0", "0", str(mixed), "1"),
                                          ("level-chunked", "0", "0", "1", None)):
        for var, val in (("QTN_FUSED_LDS_MAX", lim), ("QTN_GMEM_MAX_MACS", gmem), ("QTN_LEVEL_BUDGET", budget),
                         ("QTN_TASK_MIN", tmin)):
            if val is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, val)
        model = qaoa.MaxCut(n, e, 2, qtn.TN_C128, order="linegraph", max_sets=S)
        info = model.batch.info()
        if mode.startswith("level"):
            assert info["n_level"] == len(e) and info["n_fused"] == 0 and info["n_global"] == 0
        if mode in ("level", "level-task"):
            assert info["n_level_groups"] == 1 and info["n_level_chunked"] == 0
            assert info["n_level_tasked"] == (mode == "level-task")
        if mode.startswith("level-mixed"):
            assert info["n_level_groups"] >= 2
            assert info["n_level_tasked"] == (info["n_level_groups"] if mode == "level-mixed-task" else 0)
        if mode == "level-chunked":
            assert info["n_level_groups"] == 0 and info["n_level_chunked"] == len(e)
        if mode == "global":
            assert info["n_global"] == len(e) and info["n_fused"] == 0 and info["n_level"] == 0
        if mode == "fused":
            assert info["n_fused"] > 0
        _say(f"executor {mode} n_fused={info['n_fused']} n_global={info['n_global']} n_level={info['n_level']} "
             f"groups={info['n_level_groups']} tasked={info['n_level_tasked']} chunked={info['n_level_chunked']} launches={info['level_launches_grad']}")
        obj, grad = model.value_and_grad(ang)
        torch.cuda.synchronize()
        res[mode] = (obj.cpu().numpy(), grad.cpu().numpy())
        assert np.max(np.abs(res[mode][0] - ref)) <= 1e-12 * max(1, np.abs(ref).max())
        assert np.max(np.abs(res[mode][1] - ps)) <= 1e-10 * max(1, np.abs(ps).max())


@pytest.mark.parametrize("p", [1, 2])
def test_fused_workgroup_sizes_and_record_kernels(p, monkeypatch):
    """Every fused executor configuration gives the oracle's cost and
    gradient: one angle set per workgroup at 64, 128 and 256 lanes, and four
    angle sets per 64-lane wave. At 64 lanes the p=1 light cones run on the
    records-only kernel; the p=2 ones (intermediates of 2^12 entries, too
    large for a lane record) also need the descriptor path, and pack sets
    only as far as their LDS allows (the larger p=2 networks run on the
    global-arena executor). S = 7 leaves the last group of four sets partly
    empty."""
    qtn, qaoa = _qtn(), _qaoa()
    n = 14
    e = workloads.random_regular_graph(3, n, 8)
    S = 7
    ang = torch.tensor(workloads.qaoa_angles(11, S, p), device="cuda", dtype=torch.float64)
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    ps = np.array([gradients.parameter_shift(n, e, list(a)) for a in ang.cpu().numpy()])
    for blk, spw in ((64, 1), (128, 1), (256, 1), (64, 4)):
        monkeypatch.setenv("QTN_FUSED_BLOCK", str(blk))
        monkeypatch.setenv("QTN_SETS_PER_WAVE", str(spw))
        model = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=S)
        info = model.batch.info()
        _say(f"fused block {blk} spw {spw} p={p} rec_only={info['rec_only']} "
             f"sets={info['sets_per_wave_fwd']},{info['sets_per_wave_grad']} n_fused={info['n_fused']}")
        assert info["fused_block"] == blk and info["n_fused"] > 0
        assert info["n_fused"] + info["n_global"] + info["n_level"] == len(e)
        if p == 1 or spw == 1:
            assert info["sets_per_wave_fwd"] == info["sets_per_wave_grad"] == spw
        else:  # as many sets per wave as the largest fused program's LDS allows
            assert info["sets_per_wave_fwd"] in (1, 2, 4) and info["sets_per_wave_grad"] in (1, 2, 4)
        if blk == 64 and p == 1:
            assert info["rec_only"] == 3
        elif blk == 64:
            assert info["rec_only"] & 2 == 0
        else:
            assert info["rec_only"] == 0
        obj_f = model.expectation(ang)
        obj, grad = model.value_and_grad(ang)
        torch.cuda.synchronize()
        obj_f, obj, grad = obj_f.cpu().numpy(), obj.cpu().numpy(), grad.cpu().numpy()
        assert np.max(np.abs(obj_f - ref)) <= 1e-5 * max(1, np.abs(ref).max()), (blk, spw)
        assert np.max(np.abs(obj - ref)) <= 1e-5 * max(1, np.abs(ref).max()), (blk, spw)
        assert np.max(np.abs(grad - ps)) <= 1e-4 * max(1, np.abs(ps).max()), (blk, spw)


# --- dense regime: whole-circuit networks, large steps on the matrix cores -----------------

@pytest.mark.parametrize("d,n", [(6, 12), (5, 14)])
def test_dense_whole_circuit_mfma(d, n, monkeypatch):
    """Whole-circuit folded networks (trace on every other qubit, no light cone):
    large intermediates, complex GEMM steps on MFMA (complex64) vs the state vector."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")  # keep these networks on the level executor
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(3, 2, 1))
    S = len(ang)
    edges = e[:3]
    ref = np.array([statevector.qaoa_zz(n, e, [a[0]], [a[1]]) for a in ang])  # [set][edge]
    for dtype, tol in (("c64", 1e-5), ("c128", 1e-12)):
        dt = qtn.TN_C64 if dtype == "c64" else qtn.TN_C128
        nets = []
        for ed in edges:
            net = qaoa.edge_network(n, e, 1, ed, dtype=dt, lightcone=False)
            net.set_order(net.order_linegraph(trials=4, seed=0))
            dims = net.plan_steps()
            assert any(fx >= 6 and s >= 4 and fy >= 6 for fx, s, fy in dims), "no MFMA-sized step"
            nets.append(net)
        batch = qtn.Batch(nets, max_sets=S)
        info = batch.info()
        _say(f"dense d={d} n={n} {dtype} n_level={info['n_level']} peak={max(x.plan_info()['peak_bits'] for x in nets)}")
        out = torch.empty((len(nets), S, 2), dtype=torch.float64, device="cuda")
        batch.contract(torch.tensor(ang, device="cuda"), out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for s in range(S):
            assert np.max(np.abs(got[:, s, 0] - ref[s, :3])) < tol, (dtype, got[:, s, 0], ref[s, :3])
            assert np.max(np.abs(got[:, s, 1])) < tol


def test_autotune_keeps_results(tmp_path):
    """The autotuner changes only kernel choices: results before and after
    tuning agree, and the decisions are written to and read from its cache."""
    qtn, qaoa = _qtn(), _qaoa()
    e = workloads.random_regular_graph(6, 12, 0)
    ang = torch.tensor(workloads.qaoa_angles(4, 2, 1), device="cuda", dtype=torch.float64)
    nets = []
    for ed in e[:2]:
        net = qaoa.edge_network(12, e, 1, ed, dtype=qtn.TN_C64, lightcone=False)
        net.set_order(net.order_linegraph(trials=4, seed=0))
        nets.append(net)
    for ed in e[2:4]:
        net = qaoa.edge_network(12, e, 1, ed, dtype=qtn.TN_C64, lightcone=True)
        net.set_order(net.order_linegraph(trials=4, seed=0))
        nets.append(net)
    batch = qtn.Batch(nets, max_sets=2)
    out0 = torch.empty((len(nets), 2, 2), dtype=torch.float64, device="cuda")
    out1 = torch.empty_like(out0)
    g0 = torch.empty((len(nets), 2, 2), dtype=torch.float64, device="cuda")
    g1 = torch.empty_like(g0)
    _say("autotune before")
    batch.grad(ang, out=out0, grad_net=g0)
    torch.cuda.synchronize()
    cache = str(tmp_path / "tune.txt")
    _say("autotune run")
    batch.autotune(ang, reps=2, cache_path=cache)
    batch.grad(ang, out=out1, grad_net=g1)
    torch.cuda.synchronize()
    # against the oracle: the p=1 closed form and its derivative on every network, before and after tuning
    a = ang.cpu().numpy()
    for s in range(2):
        zz = closed_form.zz_p1(12, e, a[s, 0], a[s, 1])[:4]
        dg, db = closed_form.zz_p1_grad(12, e, a[s, 0], a[s, 1])
        g_ref = np.stack([dg[:4], db[:4]], axis=1)
        for o, g in ((out0, g0), (out1, g1)):
            assert np.max(np.abs(o.cpu().numpy()[:, s, 0] - zz)) < 1e-5
            assert np.max(np.abs(g.cpu().numpy()[:, s] - g_ref)) <= 1e-4 * max(1.0, np.abs(g_ref).max())
    text = open(cache).read()
    assert "fused_block:" in text and "mfma:" in text
    batch2 = qtn.Batch(nets, max_sets=2)
    batch2.apply_tuning(cache)
    batch2.contract(ang, out=out1)
    torch.cuda.synchronize()
    for s in range(2):
        zz = closed_form.zz_p1(12, e, a[s, 0], a[s, 1])[:4]
        assert np.max(np.abs(out1.cpu().numpy()[:, s, 0] - zz)) < 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_level_tile_shape_choices(prec, tmp_path, monkeypatch):
    """Every tile shape the tuner can choose (64 x 64, 16 x 64, 64 x 16, for
    any eligible product: a side wider than its index reads aliased entries
    and does not write them) gives the oracle's values and gradients: the
    tuner's cache is rewritten to force each shape on every matrix-core
    class of whole-circuit 6-regular n=12 p=1 networks (level executor, one
    launch per item), against the p=1 closed form and its derivative."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    monkeypatch.setenv("QTN_TASK_MIN", "1000000000")
    n = 12
    e = workloads.random_regular_graph(6, n, 0)
    ang = torch.tensor(workloads.qaoa_angles(4, 2, 1), device="cuda", dtype=torch.float64)
    nets = []
    for ed in e[:2]:
        net = qaoa.edge_network(n, e, 1, ed, dtype=qtn.TN_C64, lightcone=False)
        net.set_order(net.order_linegraph(trials=4, seed=0))
        nets.append(net)
    p_code = qtn.TN_MFMA_FP32 if prec == "fp32" else qtn.TN_MFMA_BF16X3
    batch = qtn.Batch(nets, max_sets=2)
    batch.set_precision(p_code)
    cache = str(tmp_path / "tune.txt")
    batch.autotune(ang, reps=1, cache_path=cache)
    lines = open(cache).read().splitlines()
    classes = [ln.split()[0] for ln in lines if ln.startswith("mfma:")]
    assert classes
    a = ang.cpu().numpy()
    tol_v, tol_g = (1e-5, 1e-4) if prec == "fp32" else (5e-5, 5e-4)
    for v in (2, 3, 4):
        forced = str(tmp_path / f"tile{v}.txt")
        with open(forced, "w") as f:
            for c in classes:
                f.write(f"{c} {v}\n")
        b = qtn.Batch(nets, max_sets=2)
        b.set_precision(p_code)
        b.apply_tuning(forced)
        out = torch.empty((2, 2, 2), dtype=torch.float64, device="cuda")
        gn = torch.empty((2, 2, 2), dtype=torch.float64, device="cuda")
        b.grad(ang, out=out, grad_net=gn)
        torch.cuda.synchronize()
        for s in range(2):
            zz = closed_form.zz_p1(n, e, a[s, 0], a[s, 1])[:2]
            dg, db = closed_form.zz_p1_grad(n, e, a[s, 0], a[s, 1])
            g_ref = np.stack([dg[:2], db[:2]], axis=1)
            assert np.max(np.abs(out.cpu().numpy()[:, s, 0] - zz)) < tol_v, (v, s)
            assert np.max(np.abs(gn.cpu().numpy()[:, s] - g_ref)) <= tol_g * max(1.0, np.abs(g_ref).max()), (v, s)
        _say(f"tile shape {v - 1} {prec}: ok over {len(classes)} classes")


def test_dense_split_bf16_precision():
    """Split-BF16 MFMA products on the dense whole-circuit networks: error
    against the state vector within the split's bound (at most 3 * 2^-18
    relative per product, errors of the matrix-core steps adding in
    quadrature: 5e-5 absolute on <ZZ>); FP32 products within 1e-5."""
    qtn, qaoa = _qtn(), _qaoa()
    d, n = 6, 12
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(3, 2, 1))
    ref = np.array([statevector.qaoa_zz(n, e, [a[0]], [a[1]]) for a in ang])
    nets = []
    for ed in e[:3]:
        net = qaoa.edge_network(n, e, 1, ed, dtype=qtn.TN_C64, lightcone=False)
        net.set_order(net.order_linegraph(trials=4, seed=0))
        nets.append(net)
    errs = {}
    for prec in (qtn.TN_MFMA_FP32, qtn.TN_MFMA_BF16X3):
        batch = qtn.Batch(nets, max_sets=2)
        batch.set_precision(prec)
        out = torch.empty((len(nets), 2, 2), dtype=torch.float64, device="cuda")
        _say(f"dense precision {prec}")
        batch.contract(torch.tensor(ang, device="cuda"), out=out)
        torch.cuda.synchronize()
        errs[prec] = float(np.max(np.abs(out.cpu().numpy()[:, :, 0] - ref[:, :3].T)))
    _say(f"errors {errs}")
    assert errs[qtn.TN_MFMA_FP32] < 1e-5
    assert errs[qtn.TN_MFMA_BF16X3] < 5e-5


def test_dense_whole_circuit_gradient():
    """Adjoint contraction of whole-circuit (no light cone) networks, whose
    large steps and their adjoints are matrix-core products: d<ZZ>/d(gamma, beta)
    of three edges of a 6-regular n=12 graph against the differentiated p=1
    closed form, complex64 (FP32 products) and complex128 (FP64 products)."""
    qtn, qaoa = _qtn(), _qaoa()
    d, n = 6, 12
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(6, 2, 1))
    for dt, tol_v, tol_g in ((qtn.TN_C64, 1e-5, 1e-4), (qtn.TN_C128, 1e-12, 1e-11)):
        nets = []
        for ed in e[:3]:
            net = qaoa.edge_network(n, e, 1, ed, dtype=dt, lightcone=False)
            net.set_order(net.order_linegraph(trials=4, seed=0))
            nets.append(net)
        batch = qtn.Batch(nets, max_sets=2)
        assert batch.info()["n_level"] == 3
        out = torch.empty((3, 2, 2), dtype=torch.float64, device="cuda")
        gn = torch.empty((3, 2, 2), dtype=torch.float64, device="cuda")
        _say(f"dense whole-circuit gradient dtype {dt}")
        batch.grad(torch.tensor(ang, device="cuda"), out=out, grad_net=gn)
        torch.cuda.synchronize()
        got_v, got_g = out.cpu().numpy(), gn.cpu().numpy()
        for s in range(2):
            zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])[:3]
            dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
            assert np.max(np.abs(got_v[:, s, 0] - zz)) < tol_v
            assert np.max(np.abs(got_g[:, s, 0] - dg[:3])) < tol_g, (dt, s, got_g[:, s], dg[:3], db[:3])
            assert np.max(np.abs(got_g[:, s, 1] - db[:3])) < tol_g, (dt, s, got_g[:, s], dg[:3], db[:3])


def test_split_summed_index(monkeypatch):
    """Matrix-core products with few output tiles and a long sum split their
    summed index over workgroups (partial tiles summed in range order): a
    whole-circuit 6-regular n=16 network, one parameter vector, forward and
    adjoint with splits (up to 32 ranges) and without, against the p=1 closed
    form and its derivative."""
    qtn, qaoa = _qtn(), _qaoa()
    d, n = 6, 16
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(7, 1, 1))
    zz = closed_form.zz_p1(n, e, ang[0, 0], ang[0, 1])[0]
    dg, db = closed_form.zz_p1_grad(n, e, ang[0, 0], ang[0, 1])
    res = {}
    for target in ("0", "1024"):
        monkeypatch.setenv("QTN_SPLIT_TARGET", target)
        for dt in (qtn.TN_C64, qtn.TN_C128):
            net = qaoa.edge_network(n, e, 1, e[0], dtype=dt, lightcone=False)
            net.set_order(net.order_linegraph(trials=4, seed=0))
            batch = qtn.Batch([net], max_sets=1)
            info = batch.info()
            assert (info["level_split_grad"] > 0) == (target != "0") and info["n_level"] == 1
            out = torch.empty((1, 1, 2), dtype=torch.float64, device="cuda")
            gn = torch.empty((1, 1, 2), dtype=torch.float64, device="cuda")
            _say(f"split target {target} dtype {dt}: splits fwd {info['level_split_fwd']} grad {info['level_split_grad']}")
            batch.grad(torch.tensor(ang, device="cuda"), out=out, grad_net=gn)
            torch.cuda.synchronize()
            res[(target, dt)] = (out[0, 0, 0].item(), gn[0, 0].cpu().numpy())
    for (target, dt), (v, g) in res.items():
        tol_v, tol_g = (1e-5, 1e-4) if dt == qtn.TN_C64 else (1e-12, 1e-11)
        assert abs(v - zz) < tol_v, (target, dt, v, zz)
        assert np.max(np.abs(g - np.array([dg[0], db[0]]))) < tol_g, (target, dt, g, dg[0], db[0])
    # complex128: the split changes only the order of FP64 sums
    assert abs(res[("0", qtn.TN_C128)][0] - res[("1024", qtn.TN_C128)][0]) < 1e-13


@pytest.mark.parametrize("mode", ["item", "task"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_level_mfma_tile_shapes(prec, mode, monkeypatch):
    """Matrix-core products of every tile shape (64 x 64, and 16 x 64 / 64 x 16
    where one free index has 2 to 5 bits, padded below 4; 16 x 64 with both
    narrower than 64 and a long sum, aliased columns), forward and adjoint,
    one launch per item over the networks of a group (item mode: products
    spread over many workgroups) or within one workgroup's whole program (task
    executor): 4-regular n=14 p=2 light-cone networks on the level executor,
    complex64, against the state-vector cost and the parameter-shift
    gradient."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    monkeypatch.setenv("QTN_TASK_MIN", "1" if mode == "task" else "1000000000")
    n = 14
    e = workloads.random_regular_graph(4, n, 0)
    S = 3
    ang = torch.tensor(workloads.qaoa_angles(5, S, 2), device="cuda", dtype=torch.float64)
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    ps = np.array([gradients.parameter_shift(n, e, list(a)) for a in ang.cpu().numpy()])
    model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="linegraph", max_sets=S, trials=4)
    shapes, padded = set(), 0
    for net in model.nets:
        for fx, s, fy in net.plan_steps():
            for a, ss, c in ((fx, s, fy), (fx, fy, s), (s, fx, fy)):  # the step and its two adjoints
                if ss >= 4 and min(a, c) >= 2 and (max(a, c) >= 6 or ss >= 6):
                    shapes.add((64 if a >= 6 else 16, 64 if c >= 6 or a < 6 else 16))
                    padded += min(a, c) < 4 or max(a, c) < 6  # an index narrower than its tile side
    assert shapes == {(64, 64), (16, 64), (64, 16)} and padded > 0
    model.batch.set_precision(qtn.TN_MFMA_FP32 if prec == "fp32" else qtn.TN_MFMA_BF16X3)
    info = model.batch.info()
    assert info["n_level"] == len(e) and info["n_level_groups"] == 1 and info["n_level_tasked"] == (mode == "task")
    _say(f"level mfma tiles {prec} {mode} launches fwd={info['level_launches_fwd']} grad={info['level_launches_grad']}")
    obj, grad = model.value_and_grad(ang)
    torch.cuda.synchronize()
    obj, grad = obj.cpu().numpy(), grad.cpu().numpy()
    err_c = float(np.max(np.abs(obj - ref)) / np.abs(ref).max())
    err_g = float(np.max(np.abs(grad - ps)) / np.abs(ps).max())
    _say(f"level mfma tiles {prec}: cost rel {err_c:.2e} grad rel {err_g:.2e}")
    tol_c, tol_g = (1e-5, 1e-4) if prec == "fp32" else (3e-5, 3e-4)
    assert err_c <= tol_c and err_g <= tol_g


@pytest.mark.parametrize("mode", ["item", "task"])
def test_level_mfma_fp64(mode, monkeypatch):
    """complex128 batches take their large steps on FP64 matrix-core products
    (64 x 64 tiles, FP64 accumulation): 4-regular n=14 p=2 light-cone networks
    on the level executor (item mode and task executor), forward and adjoint,
    against the state-vector cost (1e-12) and the parameter-shift gradient
    (1e-10). The precision is fixed by the dtype: FP32 / split-BF16 are
    refused for complex128 and FP64 for complex64."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    monkeypatch.setenv("QTN_TASK_MIN", "1" if mode == "task" else "1000000000")
    n = 14
    e = workloads.random_regular_graph(4, n, 0)
    S = 3
    ang = torch.tensor(workloads.qaoa_angles(6, S, 2), device="cuda", dtype=torch.float64)
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    ps = np.array([gradients.parameter_shift(n, e, list(a)) for a in ang.cpu().numpy()])
    model = qaoa.MaxCut(n, e, 2, qtn.TN_C128, order="linegraph", max_sets=S, trials=4)
    big = sum(1 for net in model.nets for fx, s, fy in net.plan_steps()
              for a, ss, c in ((fx, s, fy), (fx, fy, s), (s, fx, fy)) if ss >= 4 and a >= 6 and c >= 6)
    assert big > 0
    for bad in (qtn.TN_MFMA_FP32, qtn.TN_MFMA_BF16X3):
        with pytest.raises(qtn.QtnError):
            model.batch.set_precision(bad)
    model.batch.set_precision(qtn.TN_MFMA_FP64)
    _say(f"level mfma fp64: {big} matrix-core steps (forward and adjoint shapes)")
    obj, grad = model.value_and_grad(ang)
    torch.cuda.synchronize()
    obj, grad = obj.cpu().numpy(), grad.cpu().numpy()
    err_c = float(np.max(np.abs(obj - ref)) / np.abs(ref).max())
    err_g = float(np.max(np.abs(grad - ps)) / np.abs(ps).max())
    _say(f"level mfma fp64: cost rel {err_c:.2e} grad rel {err_g:.2e}")
    assert err_c <= 1e-12 and err_g <= 1e-10
    m64 = qaoa.MaxCut(n, e[:4], 1, qtn.TN_C64, order="linegraph", max_sets=1, trials=2)
    with pytest.raises(qtn.QtnError):
        m64.batch.set_precision(qtn.TN_MFMA_FP64)


def test_graph_replay_with_overlapping_executors(monkeypatch):
    """A batch split over the LDS fused, global-arena and level executors: the
    global-arena and level work runs on a stream forked after binding and
    joined before the combine. Eager passes and graph replays (with eager
    work between them) give identical results, and the eager result matches
    the state-vector oracle."""
    qtn, qaoa = _qtn(), _qaoa()
    n = 24
    e = workloads.random_regular_graph(3, n, 2)
    S = 4
    ang = torch.tensor(workloads.qaoa_angles(7, S, 2), device="cuda", dtype=torch.float64)
    # executor limits that split this batch three ways
    for lds, macs in ((40960, 1 << 17), (49152, 1 << 17), (32768, 1 << 18), (49152, 1 << 16)):
        monkeypatch.setenv("QTN_FUSED_LDS_MAX", str(lds))
        monkeypatch.setenv("QTN_GMEM_MAX_MACS", str(macs))
        model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="linegraph", max_sets=S, trials=2)
        info = model.batch.info()
        _say(f"overlap lds={lds} macs={macs}: fused={info['n_fused']} global={info['n_global']} level={info['n_level']}")
        if info["n_fused"] > 0 and info["n_global"] > 0 and info["n_level"] > 0:
            break
    assert info["n_fused"] > 0 and info["n_global"] > 0 and info["n_level"] > 0
    # <C> from light-cone state vectors (exact; at most 14 qubits per edge)
    ref = np.array([sum((1 - statevector.qaoa_zz_edge(n, e, a[:2], a[2:], ed)) / 2 for ed in e)
                    for a in ang.cpu().numpy()])
    obj_e, grad_e = model.value_and_grad(ang)
    torch.cuda.synchronize()
    obj_e, grad_e = obj_e.cpu().numpy(), grad_e.cpu().numpy()
    assert np.max(np.abs(obj_e - ref)) <= 1e-5 * max(1, np.abs(ref).max())
    st = torch.cuda.Stream()
    obj = torch.empty(S, dtype=torch.float64, device="cuda")
    grad = torch.empty((S, 4), dtype=torch.float64, device="cuda")
    for rep in range(3):
        _say(f"overlap graph replay {rep}")
        obj.fill_(-1.0)
        grad.fill_(-1.0)
        st.wait_stream(torch.cuda.current_stream())
        model.batch.run_graph(True, ang, obj=obj, grad=grad, stream=st)
        st.synchronize()
        assert np.array_equal(obj.cpu().numpy(), obj_e)
        assert np.array_equal(grad.cpu().numpy(), grad_e)
        o2, g2 = model.value_and_grad(ang)  # eager pass between replays
        torch.cuda.synchronize()
        assert np.array_equal(o2.cpu().numpy(), obj_e) and np.array_equal(g2.cpu().numpy(), grad_e)


def test_task_executor_matches_item_mode(monkeypatch):
    """The level executor's two launch modes on the same whole-circuit
    networks: the task executor (one launch; a workgroup runs a whole
    network program for one parameter vector) and item mode (one launch per
    op, the op spread over the chip). Both match the p=1 closed form, forward
    and gradient, for every parameter vector; more vectors than networks so
    that tasks of one network run on several workgroups at once."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")  # whole-circuit networks on the level executor
    d, n, ns = 6, 12, 5
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(3, ns, 1))
    nets = []
    for ed in e[:3]:
        net = qaoa.edge_network(n, e, 1, ed, dtype=qtn.TN_C64, lightcone=False)
        net.set_order(net.order_linegraph(trials=4, seed=0))
        nets.append(net)
    prm = torch.tensor(ang, device="cuda")
    res = {}
    for mode, task_min in (("task", "1"), ("item", "1000000000")):
        monkeypatch.setenv("QTN_TASK_MIN", task_min)
        batch = qtn.Batch(nets, max_sets=ns)
        assert batch.info()["n_level"] == 3
        out = torch.zeros((3, ns, 2), dtype=torch.float64, device="cuda")
        gn = torch.zeros((3, ns, 2), dtype=torch.float64, device="cuda")
        _say(f"level executor {mode} mode, 3 nets, {ns} sets")
        batch.grad(prm, out=out, grad_net=gn)
        torch.cuda.synchronize()
        o, g = out.cpu().numpy(), gn.cpu().numpy()
        for s in range(ns):
            zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])[:3]
            dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
            assert np.max(np.abs(o[:, s, 0] - zz)) < 1e-5
            assert np.max(np.abs(g[:, s, 0] - dg[:3])) <= 1e-4 * max(1.0, np.abs(dg[:3]).max())
            assert np.max(np.abs(g[:, s, 1] - db[:3])) <= 1e-4 * max(1.0, np.abs(db[:3]).max())
        res[mode] = (o, g)
    assert np.max(np.abs(res["task"][0] - res["item"][0])) < 1e-5


def test_task_executor_lds_residency(monkeypatch):
    """The task executor keeps a program's small tensors (and a mirror of its
    leaves) in LDS, takes small summed-index offsets from packed bit
    positions, and runs small contractions whose operands are all in LDS
    from lane records on one wave: 4-regular n=14 p=2 light-cone networks,
    forward + adjoint, agree with that arena switched off (every tensor in
    the region, every offset from its table; the lane records sum some
    entries in another order, so to complex64 rounding) and match the
    state-vector cost and parameter-shift gradient."""
    qtn, qaoa = _qtn(), _qaoa()
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "0")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", "0")
    monkeypatch.setenv("QTN_TASK_MIN", "1")
    n = 14
    e = workloads.random_regular_graph(4, n, 0)
    S = 3
    ang = torch.tensor(workloads.qaoa_angles(12, S, 2), device="cuda", dtype=torch.float64)
    ref = np.array([gradients.cost(n, e, list(a)) for a in ang.cpu().numpy()])
    ps = np.array([gradients.parameter_shift(n, e, list(a)) for a in ang.cpu().numpy()])
    res = {}
    for lds in ("default", "0"):
        if lds == "0":
            monkeypatch.setenv("QTN_TASK_LDS", "0")
        model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="linegraph", max_sets=S, trials=4)
        assert model.batch.info()["n_level_tasked"] == 1
        _say(f"task executor LDS arena {lds}")
        obj, grad = model.value_and_grad(ang)
        torch.cuda.synchronize()
        res[lds] = (obj.cpu().numpy(), grad.cpu().numpy())
    assert np.max(np.abs(res["default"][0] - res["0"][0])) <= 1e-6 * np.abs(res["0"][0]).max()
    assert np.max(np.abs(res["default"][1] - res["0"][1])) <= 1e-5 * np.abs(res["0"][1]).max()
    obj, grad = res["default"]
    assert np.max(np.abs(obj - ref)) <= 1e-5 * np.abs(ref).max()
    assert np.max(np.abs(grad - ps)) <= 1e-4 * np.abs(ps).max()


def test_global_arena_networks_join_task_executor(monkeypatch):
    """When a batch's level networks are many enough for the task executor,
    the networks the global-arena executor would take run there too: the
    3-way split batch (3-regular n=24 p=2 under lowered executor limits)
    with the task threshold at one pair puts every non-LDS network on the
    level executor, and matches the same batch with the global-arena
    executor kept."""
    qtn, qaoa = _qtn(), _qaoa()
    n = 24
    e = workloads.random_regular_graph(3, n, 2)
    S = 4
    ang = torch.tensor(workloads.qaoa_angles(13, S, 2), device="cuda", dtype=torch.float64)
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "32768")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", str(1 << 18))
    monkeypatch.setenv("QTN_TASK_MIN", "1")
    res = {}
    for join in ("0", "1"):
        monkeypatch.setenv("QTN_GMEM_JOIN", join)
        model = qaoa.MaxCut(n, e, 2, qtn.TN_C64, order="linegraph", max_sets=S, trials=2)
        info = model.batch.info()
        if join == "1":
            assert info["n_global"] == 0 and info["n_level"] == len(e) - info["n_fused"]
        else:
            assert info["n_global"] > 0
        _say(f"global-arena join {join}: fused={info['n_fused']} global={info['n_global']} level={info['n_level']}")
        obj, grad = model.value_and_grad(ang)
        torch.cuda.synchronize()
        res[join] = (obj.cpu().numpy(), grad.cpu().numpy())
    assert np.max(np.abs(res["0"][0] - res["1"][0])) <= 1e-5 * np.abs(res["0"][0]).max()
    assert np.max(np.abs(res["0"][1] - res["1"][1])) <= 1e-4 * np.abs(res["0"][1]).max()


def test_gradient_recompute_under_memory_limit():
    """Forward runs recomputed before their adjoints (a memory limit below
    what the gradient program needs with every forward intermediate kept)
    give the same gradient: complex128 whole-circuit network of a 4-regular
    n=10 p=2 edge, on the one-network path and in a batch of two angle sets,
    against the plan without recomputation (1e-12) and the parameter-shift
    rule on the edge's light cone (1e-10)."""
    qtn, qaoa = _qtn(), _qaoa()
    n, p = 10, 2
    e = workloads.random_regular_graph(4, n, 0)
    ang = np.array(workloads.qaoa_angles(3, 2, p))
    full = qaoa.edge_network(n, e, p, e[0], dtype=qtn.TN_C128, lightcone=False)
    pi = full.order_linegraph(trials=8, seed=0)
    full.set_order(pi)
    cut = qaoa.edge_network(n, e, p, e[0], dtype=qtn.TN_C128, lightcone=False)
    cut.set_memory_limit(int(full.plan_info()["grad_bytes"] * 0.8))
    cut.set_order(pi)
    runs = cut.plan_info()["recompute_runs"]
    _say(f"recompute runs {runs}")
    assert runs > 1
    for a in ang:
        ps = gradients.parameter_shift_edge(n, e, list(a), e[0])
        v0, g0 = full.grad(a)
        v1, g1 = cut.grad(a)
        assert abs(v1 - v0) < 1e-12 and np.max(np.abs(g1 - g0)) < 1e-12, (v0, v1, g0, g1)
        assert np.max(np.abs(g1 - ps)) < 1e-10, (g1, ps)
    b = qtn.Batch([cut], max_sets=2)
    out = torch.empty((1, 2, 2), dtype=torch.float64, device="cuda")
    gn = torch.empty((1, 2, 2 * p), dtype=torch.float64, device="cuda")
    b.grad(torch.tensor(ang, device="cuda"), out=out, grad_net=gn)
    torch.cuda.synchronize()
    for s, a in enumerate(ang):
        ps = gradients.parameter_shift_edge(n, e, list(a), e[0])
        assert np.max(np.abs(gn[0, s].cpu().numpy() - ps)) < 1e-10
