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


@pytest.mark.parametrize("d,n", [(4, 50), (4, 70), (4, 100), (5, 50), (5, 70), (5, 100)])
@pytest.mark.parametrize("p", [1, 2])
def test_config3_batched_graphs(d, n, p):
    """All edge networks x 64 angle sets per graph, complex64, one batched pass."""
    from paper_1709_03636_amd import qtn, qaoa
    e = workloads.random_regular_graph(d, n, 0)
    S = 64
    ang = np.array(workloads.qaoa_angles(0, S, p))
    model = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=S, trials=4)
    info = model.batch.info()
    _say(f"config3 d={d} n={n} p={p} nets={len(e)} fused={info['n_fused']} global={info['n_global']} level={info['n_level']}")
    out = torch.empty((len(e), S, 2), dtype=torch.float64, device="cuda")
    obj = model.expectation(torch.tensor(ang, device="cuda"), out=out)
    torch.cuda.synchronize()
    o, ob = out.cpu().numpy(), obj.cpu().numpy()
    assert np.all(np.abs(o[..., 0]) <= 1 + 1e-5)
    assert np.max(np.abs(o[..., 1])) < 1e-5
    assert np.all((ob >= -1e-5) & (ob <= len(e) + 1e-5))
    np.testing.assert_allclose(ob, np.sum((1 - o[..., 0]) / 2, axis=0), rtol=1e-12, atol=1e-9)
    if p == 1:
        for s in range(S):
            zz = closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1])
            assert np.max(np.abs(o[:, s, 0] - zz)) < 1e-5
    else:
        rng = workloads.SplitMix64(d * 1000 + n)
        for _ in range(6):
            i, s = rng.below(len(e)), rng.below(S)
            ref = _oracle_tn_zz(n, e, ang[s], p, e[i])
            assert abs(o[i, s, 0] - ref.real) < 1e-5, (i, s, o[i, s, 0], ref)


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
    and the batched pass, all against the closed form."""
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
