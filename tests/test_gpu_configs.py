"""GPU parity at the full sizes of the benchmark configurations.

Each configuration runs through the batched C-ABI path at its full size;
outputs are checked against the FP64 oracle wherever the oracle computes
them one by one (closed form for p = 1, light-cone state vectors, the plain
tensor-network contraction on light cones for p = 2), and against properties
that hold at any size elsewhere (|<ZZ>| <= 1, Im <ZZ> = 0, 0 <= <C> <= |E|).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import closed_form, gates, gradients, statevector, tensornet

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
    qtn.lib()


def _oracle_tn_zz(n, e, ang, p, edge):
    gl = gates.qaoa_gate_list(n, e, ang[:p], ang[p:])[n:]
    plus = [np.array([1.0, 1.0]) / np.sqrt(2.0)] * n
    pauli = [0] * n
    pauli[edge[0]] = pauli[edge[1]] = 3
    return tensornet.expectation(n, gl, pauli, init=plus, lightcone=True)


# Tolerances of the split-BF16 matrix-core path (complex64 operands split as
# x = hi + lo in bfloat16, products hi*hi + hi*lo + lo*hi, FP32 accumulation).
# Each real product then carries a relative error of at most 3 * 2^-18 (the
# rounding of lo and the dropped lo*lo term, 2^-18 each) instead of FP32's
# 2^-24; with errors of independent steps adding in quadrature over at most
# 20 matrix-core steps on a network's path (sqrt(20) ~ 4.5) the value error
# stays below 3 * 2^-18 * 4.5 ~ 5e-5. <Z_u Z_v> is on the scale of Tr rho = 1,
# so the bound is absolute there; <C> relative; gradients, as in FP32, ten
# times the value bound times max(1, |g|).
TOL_ZZ_BF16, TOL_C_BF16, TOL_G_BF16 = 5e-5, 5e-5, 5e-4
GRID_TRIALS = {1: 4, 2: 128}  # line-graph order restarts per network (as the benchmark plans them)


def _golden_p2():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config3_p2.json")
    return {(g["d"], g["n"]): g for g in json.load(open(path))["graphs"]}


@pytest.mark.parametrize("d,n", [(4, 50), (4, 70), (4, 100), (5, 50), (5, 70), (5, 100)])
@pytest.mark.parametrize("p", [1, 2])
def test_config3_timed_path(d, n, p):
    """The batching configuration as timed: all edge networks x 64 angle sets,
    split-BF16 matrix-core products, autotuned, forward + adjoint gradient
    replayed twice from the captured graph. The replayed values and gradients
    are checked: p = 1 against the closed form and its derivative on every
    edge and set; p = 2 against the oracle's light-cone contraction on 64
    sampled (edge, set) pairs and the parameter-shift rule on 4 of them
    (tests/golden/config3_p2.json); both replays agree bit for bit."""
    from paper_1709_03636_amd import qtn, qaoa
    e = workloads.random_regular_graph(d, n, 0)
    S, m = 64, len(e)
    ang = np.array(workloads.qaoa_angles(0, S, p))
    model = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=S, trials=GRID_TRIALS[p])
    model.batch.set_precision(qtn.TN_MFMA_BF16X3)
    st = torch.cuda.Stream()
    prm = torch.tensor(ang, device="cuda")
    model.batch.autotune(prm, reps=2, stream=st)
    info = model.batch.info()
    _say(f"config3 d={d} n={n} p={p} nets={m} fused={info['n_fused']} global={info['n_global']} level={info['n_level']}")
    out = torch.empty((m, S, 2), dtype=torch.float64, device="cuda")
    gnet = torch.empty((m, S, 2 * p), dtype=torch.float64, device="cuda")
    obj = torch.empty(S, dtype=torch.float64, device="cuda")
    grad = torch.empty((S, 2 * p), dtype=torch.float64, device="cuda")
    reps = []
    for _ in range(2):
        model.batch.run_graph(True, prm, out=out, obj=obj, grad=grad, grad_net=gnet, stream=st)
        st.synchronize()
        reps.append([t.cpu().numpy().copy() for t in (out, gnet, obj, grad)])
    for a, b in zip(reps[0], reps[1]):
        assert np.array_equal(a, b), "graph replays differ"
    o, gn, ob, gr = reps[1]
    assert np.all(np.isfinite(o)) and np.all(np.isfinite(gn))
    assert np.max(np.abs(o[..., 1])) < TOL_ZZ_BF16
    np.testing.assert_allclose(ob, m / 2 - 0.5 * o[..., 0].sum(axis=0), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(gr, -0.5 * gn.sum(axis=0), rtol=1e-12, atol=1e-9)
    if p == 1:
        for s in range(S):
            zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
            dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
            assert np.max(np.abs(o[:, s, 0] - zz)) < TOL_ZZ_BF16, s
            c_ref = float(np.sum((1 - zz) / 2))
            assert abs(ob[s] - c_ref) <= TOL_C_BF16 * c_ref, (s, ob[s], c_ref)
            g_e = np.stack([dg, db], axis=1)
            assert np.max(np.abs(gn[:, s] - g_e)) <= TOL_G_BF16 * max(1.0, np.abs(g_e).max()), s
            g_ref = -0.5 * g_e.sum(axis=0)
            assert np.max(np.abs(gr[s] - g_ref)) <= TOL_G_BF16 * max(1.0, np.abs(g_ref).max()), (s, gr[s], g_ref)
    else:
        gold = _golden_p2()[(d, n)]
        err = 0.0
        for i, s, v in gold["values"]:
            err = max(err, abs(o[i, s, 0] - v))
        _say(f"config3 d={d} n={n} p=2 max |dZZ| over {len(gold['values'])} sampled pairs: {err:.2e}")
        assert err < TOL_ZZ_BF16
        for i, s, g in gold["grads"]:
            g = np.array(g)
            assert np.max(np.abs(gn[i, s] - g)) <= TOL_G_BF16 * max(1.0, np.abs(g).max()), (i, s, gn[i, s], g)


def test_config4_gradient_n60_p2():
    """QAOA p=2, 3-regular n=60: <C> and its adjoint gradient (complex64) against
    light-cone state vectors, the parameter-shift rule and finite differences."""
    from paper_1709_03636_amd import qtn, qaoa
    n, p = 60, 2
    e = workloads.random_regular_graph(3, n, 0)
    S = 3
    ang = np.array(workloads.qaoa_angles(0, S, p))
    model = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=S)
    _say(f"config4 n={n} p={p} nets={len(e)} info={model.batch.info()}")
    out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    obj, grad = model.value_and_grad(torch.tensor(ang, device="cuda"), out=out)
    torch.cuda.synchronize()
    o, ob, gr = out.cpu().numpy(), obj.cpu().numpy(), grad.cpu().numpy()
    for s in range(S):
        zz = np.array([statevector.qaoa_zz_edge(n, e, ang[s, :p], ang[s, p:], ed) for ed in e])
        assert np.max(np.abs(o[:, s, 0] - zz)) < 1e-5
        c_ref = float(np.sum((1 - zz) / 2))
        assert abs(ob[s] - c_ref) <= 1e-5 * c_ref
    s = 1
    ps = sum(-0.5 * gradients.parameter_shift_edge(n, e, ang[s], ed) for ed in e)
    assert np.max(np.abs(gr[s] - ps)) <= 1e-4 * max(1.0, np.abs(ps).max()), (gr[s], ps)
    h = 1e-4
    fd = np.zeros(2 * p)
    for k in range(2 * p):
        dp = np.zeros(2 * p)
        dp[k] = h
        cp = sum((1 - statevector.qaoa_zz_edge(n, e, (ang[s] + dp)[:p], (ang[s] + dp)[p:], ed)) / 2 for ed in e)
        cm = sum((1 - statevector.qaoa_zz_edge(n, e, (ang[s] - dp)[:p], (ang[s] - dp)[p:], ed)) / 2 for ed in e)
        fd[k] = (cp - cm) / (2 * h)
    assert np.max(np.abs(fd - ps)) <= 1e-5 * max(1.0, np.abs(ps).max())
    assert np.max(np.abs(gr[s] - fd)) <= 1e-4 * max(1.0, np.abs(fd).max())


def test_config2_plain_and_batched_agree():
    """3-regular n=100 p=1: one network per launch (complex64 and complex128)
    and the batched pass over the same networks (64 angle sets, graph
    replay), all against the closed form."""
    from paper_1709_03636_amd import qtn, qaoa
    n = 100
    e = workloads.random_regular_graph(3, n, 0)
    a = np.array(workloads.qaoa_angles(0, 1, 1))[0]
    zz = closed_form.zz_p1(n, e, a[0], a[1])
    for dt, tol in ((qtn.TN_C64, 1e-5), (qtn.TN_C128, 1e-12)):
        nets = qaoa.edge_networks(n, e, 1, dt, order="linegraph", trials=4)
        _say(f"config2 plain dtype={dt}")
        got = np.array([net.contract(a).real for net in nets])
        assert np.max(np.abs(got - zz)) < tol
        S = 64
        ang = np.array(workloads.qaoa_angles(0, S, 1))
        ang[0] = a
        batch = qtn.Batch(nets, coef=[-0.5] * len(e), offset=0.5 * len(e), max_sets=S)
        st = torch.cuda.Stream()
        prm = torch.tensor(ang, device="cuda")
        out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
        obj = torch.empty(S, dtype=torch.float64, device="cuda")
        _say(f"config2 batched dtype={dt}")
        for _ in range(2):
            batch.run_graph(False, prm, out=out, obj=obj, stream=st)
        st.synchronize()
        o, ob = out.cpu().numpy(), obj.cpu().numpy()
        assert np.array_equal(o[:, 0, 0], got), "batched and one-network-per-launch results differ"
        for s in range(S):
            z = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
            assert np.max(np.abs(o[:, s, 0] - z)) < tol
            c = float(np.sum((1 - z) / 2))
            assert abs(ob[s] - c) <= tol * c


def test_headline_timed_path():
    """The 3-regular n=100 p=1 batch (150 networks x 64 angle sets, complex64)
    as the benchmark times it: autotuned, forward + gradient replayed from the
    captured graph; every replayed <Z_u Z_v>, <C> and gradient entry against
    the closed form and its derivative."""
    from paper_1709_03636_amd import qtn, qaoa
    n, S = 100, 64
    e = workloads.random_regular_graph(3, n, 0)
    ang = np.array(workloads.qaoa_angles(0, S, 1))
    model = qaoa.MaxCut(n, e, 1, qtn.TN_C64, order="linegraph", max_sets=S, trials=4)
    st = torch.cuda.Stream()
    prm = torch.tensor(ang, device="cuda")
    model.batch.autotune(prm, reps=3, stream=st)
    out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    gnet = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    obj = torch.empty(S, dtype=torch.float64, device="cuda")
    grad = torch.empty((S, 2), dtype=torch.float64, device="cuda")
    for _ in range(3):
        model.batch.run_graph(True, prm, out=out, obj=obj, grad=grad, grad_net=gnet, stream=st)
    st.synchronize()
    o, gn, ob, gr = (t.cpu().numpy() for t in (out, gnet, obj, grad))
    for s in range(S):
        zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
        dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
        assert np.max(np.abs(o[:, s, 0] - zz)) < 1e-5
        c = float(np.sum((1 - zz) / 2))
        assert abs(ob[s] - c) <= 1e-5 * c
        g_e = np.stack([dg, db], axis=1)
        assert np.max(np.abs(gn[:, s] - g_e)) <= 1e-4 * max(1.0, np.abs(g_e).max())
        g_ref = -0.5 * g_e.sum(axis=0)
        assert np.max(np.abs(gr[s] - g_ref)) <= 1e-4 * max(1.0, np.abs(g_ref).max())


def test_autograd_function_backward():
    """torch.autograd.Function around the batched pass: params.grad after
    backward of a weighted sum equals the weights times the adjoint gradient,
    which equals the closed-form derivative of <C>."""
    from paper_1709_03636_amd import qtn, qaoa
    n, S = 12, 3
    e = workloads.random_regular_graph(3, n, 0)
    model = qaoa.MaxCut(n, e, 1, qtn.TN_C64, order="stochastic", seed=0, max_sets=S)
    ang = np.array(workloads.qaoa_angles(5, S, 1))
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    QAOAExpectation = qaoa.make_autograd()
    x = torch.tensor(ang, device="cuda", requires_grad=True)
    val = QAOAExpectation.apply(x, model)
    (val * w).sum().backward()
    torch.cuda.synchronize()
    obj_ref, grad_ref = model.value_and_grad(torch.tensor(ang, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(val.detach(), obj_ref)
    assert torch.equal(x.grad, w.reshape(-1, 1) * grad_ref)
    for s in range(S):
        dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
        g = np.array([-0.5 * dg.sum(), -0.5 * db.sum()])
        assert np.max(np.abs(x.grad[s].cpu().numpy() / w[s].item() - g)) <= 1e-4 * max(1.0, np.abs(g).max())


def test_config5_whole_circuit_2p30():
    """The dense regime at its stated size: the whole-circuit folded network
    of edge 0 of the seeded 5-regular n=30 graph at p=1 (no light cone),
    line-graph order from 1024 restarts (largest intermediate 2^30 entries,
    8 GiB complex64; 4.5e13 flops forward), on the level executor with FP32
    and split-BF16 matrix-core products. <Z_u Z_v> and its gradient against
    the p=1 closed form: 1e-6 / 1e-5 absolute (FP32), 1e-5 / 1e-4 (split
    BF16). Exercises element offsets past 2^31 in the set's region."""
    from paper_1709_03636_amd import qtn, qaoa
    d, n = 5, 30
    e = workloads.random_regular_graph(d, n, 0)
    a0 = np.array(workloads.qaoa_angles(0, 64, 1))[0]
    zz = closed_form.zz_p1(n, e, a0[0], a0[1])[0]
    dg, db = closed_form.zz_p1_grad(n, e, a0[0], a0[1])
    net = qaoa.edge_network(n, e, 1, e[0], dtype=qtn.TN_C64, lightcone=False)
    net.set_order(net.order_linegraph(trials=1024, seed=0))
    info = net.plan_info()
    assert info["peak_bits"] == 30
    prm = torch.tensor(np.array([a0]), dtype=torch.float64, device="cuda")
    for prec, tz, tg in ((qtn.TN_MFMA_FP32, 1e-6, 1e-5), (qtn.TN_MFMA_BF16X3, 1e-5, 1e-4)):
        b = qtn.Batch([net], max_sets=1)
        b.set_precision(prec)
        assert b.workspace_bytes() > 8 << 31  # the region passes 2^31 elements
        out = torch.empty((1, 1, 2), dtype=torch.float64, device="cuda")
        gn = torch.empty((1, 1, 2), dtype=torch.float64, device="cuda")
        _say(f"config 5 whole circuit d={d} n={n} 2^30, precision {prec}: forward")
        b.contract(prm, out=out)
        torch.cuda.synchronize()
        v = out[0, 0].cpu().numpy()
        assert abs(v[0] - zz) <= tz and abs(v[1]) <= tz
        _say(f"config 5 precision {prec}: forward + gradient")
        b.grad(prm, out=out, grad_net=gn)
        torch.cuda.synchronize()
        g = gn[0, 0].cpu().numpy()
        assert abs(out[0, 0, 0].item() - zz) <= tz
        assert abs(g[0] - dg[0]) <= tg and abs(g[1] - db[0]) <= tg
        del b
        torch.cuda.empty_cache()
