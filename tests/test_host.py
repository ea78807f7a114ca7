"""Host-side logic of the C-ABI library (no GPU calls): exports, network
construction, light cone, orders (Algorithms 1 and 2), plan shapes and
error paths."""
import itertools
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def qtn():
    from paper_1709_03636_amd import qtn as q
    q.lib()
    return q


@pytest.fixture(scope="module")
def qaoa():
    from paper_1709_03636_amd import qaoa as m
    return m


def test_library_exports_every_declared_symbol(qtn):
    hdr = open(os.path.join(ROOT, "include", "qtn.h")).read()
    names = set(re.findall(r"^\s*(?:int64_t|int|void|const char \*)\s*(tn_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 20
    L = qtn.lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert b"gfx950" in L.tn_version()


def test_binding_structs_match_header(qtn):
    """Every struct the header declares has a ctypes twin with the same
    fields in the same order, of the same C types (so the same layout)."""
    import ctypes
    hdr = open(os.path.join(ROOT, "include", "qtn.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    cmap = {"int32_t": ctypes.c_int32, "double": ctypes.c_double, "uint64_t": ctypes.c_uint64}
    structs = re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", hdr, re.S)
    assert {n for _, n in structs} >= {"tn_gate", "tn_target", "tn_plan_stats", "tn_batch_stats"}
    for body, name in structs:
        fields = []
        for decl in filter(None, (d.strip() for d in body.split(";"))):
            m = re.match(r"(const\s+)?(\w+)\s*(\*?)\s*(.*)", decl)
            ctype, ptr = m.group(2), m.group(3)
            for nm in (x.strip().lstrip("*").strip() for x in m.group(4).split(",")):
                arr = re.match(r"(\w+)\[(\d+)\]$", nm)
                fields.append((arr.group(1) if arr else nm, ctype, bool(ptr) or m.group(4).lstrip().startswith("*"),
                               int(arr.group(2)) if arr else 0))
        py = getattr(qtn, name)._fields_
        assert [f[0] for f in fields] == [f[0] for f in py], name
        for (nm, ctype, ptr, n_arr), (_, pt) in zip(fields, py):
            if ptr:
                assert issubclass(pt, ctypes._Pointer), (name, nm)
            elif n_arr:
                assert issubclass(pt, ctypes.Array) and pt._length_ == n_arr and pt._type_ is cmap[ctype], (name, nm)
            else:
                assert pt is cmap[ctype], (name, nm)


def test_qaoa_p1_network_shape(qtn, qaoa):
    # triangle-free edge of a 3-regular graph: 6 boundary vectors, 5 ZZ, 2 RX, 6 measurements
    e = workloads.random_regular_graph(3, 100, 0)
    net = qaoa.edge_network(100, e, 1, e[0])
    nw, nt, ends = net.wires()
    assert (nt, nw) == (19, 18)
    # closed network: every wire joins two distinct tensors
    assert np.all(ends >= 0) and np.all(ends[:, 0] != ends[:, 1])


def test_lightcone_off_keeps_everything(qtn, qaoa):
    e = workloads.random_regular_graph(3, 8, 1)
    net = qaoa.edge_network(8, e, 1, e[0], lightcone=False)
    nw, nt, _ = net.wires()
    assert nt == 8 + len(e) + 8 + 8


def test_stochastic_order_is_permutation_and_deterministic(qtn, qaoa):
    e = workloads.random_regular_graph(3, 20, 3)
    net = qaoa.edge_network(20, e, 2, e[4])
    a = net.order_stochastic(7)
    b = net.order_stochastic(7)
    c = net.order_stochastic(8)
    assert sorted(a) == list(range(net.n_wires))
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def _simulate_alg2_costs(ends, n_tensors, pi):
    """Replays an order at the wire level and returns the cost of each merge."""
    tw = [set() for _ in range(n_tensors)]
    for w, (x, y) in enumerate(ends):
        tw[x].add(w)
        tw[y].add(w)
    owner = {w: [x, y] for w, (x, y) in enumerate(ends)}
    costs = []
    for w in pi:
        a, b = owner[w]
        if a == b:
            continue
        sh = tw[a] & tw[b]
        rc = len(tw[a]) + len(tw[b]) - 2 * len(sh)
        costs.append(rc - max(len(tw[a]), len(tw[b])))
        new = (tw[a] | tw[b]) - sh
        tw.append(new)
        nid = len(tw) - 1
        for x in tw[a] | tw[b]:
            owner[x] = [nid if t in (a, b) else t for t in owner[x]]
    return costs


def test_stochastic_order_prefers_cheap_merges(qtn, qaoa):
    """Alg. 2 accepts a merge only when its cost is <= the threshold, which
    restarts at -1 after every acceptance: the first merge must have cost -1
    (a boundary vector absorbed), and most merges are non-increasing."""
    e = workloads.random_regular_graph(4, 20, 2)
    net = qaoa.edge_network(20, e, 2, e[0])
    nw, nt, ends = net.wires()
    pi = net.order_stochastic(0)
    costs = _simulate_alg2_costs(ends, nt, pi)
    assert costs[0] == -1
    assert sum(c <= 0 for c in costs) >= 0.7 * len(costs)


def test_linegraph_order_quality(qtn, qaoa):
    e = workloads.random_regular_graph(5, 50, 0)
    net = qaoa.edge_network(50, e, 2, e[0])
    pi = net.order_linegraph(trials=4, seed=1)
    assert sorted(pi) == list(range(net.n_wires))
    net.set_order(pi)
    lg = net.plan_info()
    # min-fill on the line graph keeps the peak far below the full light cone
    assert lg["peak_bits"] <= 20
    assert lg["n_steps"] == lg["n_tensors"] - lg["n_components"]


def test_linegraph_restarts_and_threads(qtn, qaoa):
    """More restarts of the line-graph search never give a worse order by its
    (peak, flops) key, and networks ordered on host threads get the same
    orders as built one after another."""
    e = workloads.random_regular_graph(5, 30, 0)
    key = {}
    for trials in (4, 32):
        net = qaoa.edge_network(30, e, 2, e[3])
        net.set_order(net.order_linegraph(trials=trials, seed=0))
        pi = net.plan_info()
        key[trials] = (pi["peak_bits"], pi["flops"])
    assert key[32] <= key[4]
    seq = qaoa.edge_networks(30, e[:10], 2, order="linegraph", trials=8, workers=1)
    par = qaoa.edge_networks(30, e[:10], 2, order="linegraph", trials=8, workers=4)
    for a, b in zip(seq, par):
        assert np.array_equal(a.plan_steps(), b.plan_steps())


def test_gradient_recompute_plan_under_memory_limit(qtn, qaoa):
    """A memory limit below what the gradient program needs (it keeps every
    forward intermediate) makes tn_set_order cut the forward steps into runs
    that are recomputed before their adjoints: the gradient program then fits
    the limit, the forward program is unchanged, and a generous limit leaves
    the plan without recomputation."""
    n, p = 10, 2
    e = workloads.random_regular_graph(4, n, 0)
    net = qaoa.edge_network(n, e, p, e[0], dtype=qtn.TN_C128, lightcone=False)
    pi = net.order_linegraph(trials=8, seed=0)
    net.set_order(pi)
    full = net.plan_info()
    assert full["recompute_runs"] == 1 and full["grad_bytes"] > full["peak_live_bytes"]
    for frac, expect_runs in ((0.8, True), (1.5, False)):
        limit = int(full["grad_bytes"] * frac)
        small = qaoa.edge_network(n, e, p, e[0], dtype=qtn.TN_C128, lightcone=False)
        small.set_memory_limit(limit)
        small.set_order(pi)
        info = small.plan_info()
        assert (info["recompute_runs"] > 1) == expect_runs, (frac, info["recompute_runs"])
        assert info["grad_bytes"] <= limit
        for k in ("flops", "bytes", "peak_live_bytes", "n_steps", "peak_bits"):
            assert info[k] == full[k], k
    # below what any cut reaches, the order still stands (the forward fits)
    tight = qaoa.edge_network(n, e, p, e[0], dtype=qtn.TN_C128, lightcone=False)
    tight.set_memory_limit(int(full["peak_live_bytes"] * 1.01))
    tight.set_order(pi)
    assert tight.plan_info()["recompute_runs"] > 1


def test_plan_shapes_and_flops(qtn, qaoa):
    """Eq. (1): C has rank x+z and costs m^(x+y+z) multiply-adds (m = 4 per wire = 2 bits)."""
    e = workloads.random_regular_graph(3, 12, 0)
    net = qaoa.edge_network(12, e, 1, e[0])
    net.set_order(net.order_stochastic(0))
    info = net.plan_info()
    dims = net.plan_steps()
    assert len(dims) == info["n_steps"] == 18
    flops = sum(8.0 * 2 ** int(d.sum()) for d in dims)
    assert flops == info["flops"]
    byts = sum(8.0 * (2 ** int(d[0] + d[1]) + 2 ** int(d[1] + d[2]) + 2 ** int(d[0] + d[2])) for d in dims)
    assert byts == info["bytes"]
    assert info["peak_bits"] == max(int(d[0] + d[2]) for d in dims)
    assert np.all(dims % 2 == 0)  # folded network: whole wires only
    assert dims[-1][0] == 0 and dims[-1][2] == 0  # last step: scalar


def test_error_paths(qtn):
    with pytest.raises(qtn.QtnError) as ei:
        qtn.Network(2, [("ZZ", 0, 0, -1, 0.3)], qtn.TN_EXPECTATION, [3, 3])
    assert ei.value.code == qtn.TN_EINVAL
    with pytest.raises(qtn.QtnError) as ei:
        qtn.Network(2, [("RX", 5, -1, -1, 0.3)], qtn.TN_EXPECTATION, [3, 3])
    assert ei.value.code == qtn.TN_EINVAL
    with pytest.raises(qtn.QtnError) as ei:
        qtn.Network(2, [("RX", 0, -1, 3, 0.3)], qtn.TN_EXPECTATION, [3, 3], n_params=2)
    assert ei.value.code == qtn.TN_EINVAL
    net = qtn.Network(2, [("H", 0, -1, -1, 0.0), ("CNOT", 0, 1, -1, 0.0)], qtn.TN_EXPECTATION, [3, 3])
    nw = net.n_wires
    with pytest.raises(qtn.QtnError) as ei:
        net.set_order([0] * nw)
    assert ei.value.code == qtn.TN_EORDER
    with pytest.raises(qtn.QtnError) as ei:
        net.set_order(list(range(nw - 1)))
    assert ei.value.code == qtn.TN_EORDER
    with pytest.raises(qtn.QtnError) as ei:
        net.plan_info()
    assert ei.value.code == qtn.TN_EORDER
    net.set_memory_limit(16)
    with pytest.raises(qtn.QtnError) as ei:
        net.set_order(net.order_stochastic(0))
    assert ei.value.code == qtn.TN_ENOMEM
    net.set_memory_limit(1 << 30)
    net.set_order(net.order_stochastic(0))
    assert net.plan_info()["n_steps"] > 0


def test_parallel_wires_are_contracted_once(qtn):
    # two gates on the same pair of qubits create tensors joined by two wires
    gates = [("CNOT", 0, 1, -1, 0.0), ("CZ", 0, 1, -1, 0.0), ("H", 0, -1, -1, 0.0)]
    net = qtn.Network(2, gates, qtn.TN_EXPECTATION, [3, 1], lightcone=False)
    nw, nt, _ = net.wires()
    for seed in range(5):
        net.set_order(net.order_stochastic(seed))
        info = net.plan_info()
        assert info["n_steps"] == nt - info["n_components"]
    net.set_order(list(range(nw))[::-1])
    assert net.plan_info()["n_steps"] == nt - net.plan_info()["n_components"]


def test_disconnected_components(qtn):
    # no two-qubit gates: every qubit is its own component
    gates = [("RX", q, -1, -1, 0.1 * (q + 1)) for q in range(3)]
    net = qtn.Network(3, gates, qtn.TN_EXPECTATION, [3, 0, 1], lightcone=False)
    net.set_order(net.order_linegraph(trials=1))
    assert net.plan_info()["n_components"] == 3


def test_channel_gates_light_cone_and_errors(qtn):
    """A trace-preserving channel outside the light cone is dropped like a
    unitary gate; a map that is not trace preserving turns the cone off;
    channels are rejected in the (unfolded) amplitude mode."""
    from paper_1709_03636_amd import noise
    base = [("H", 0, -1, -1, 0.0), ("CNOT", 0, 1, -1, 0.0), ("H", 2, -1, -1, 0.0)]
    tp = base + [noise.channel_gate(noise.depolarizing(0.1), 2)]
    ntp = base + [noise.channel_gate([np.diag([1.0, 0.0])], 2)]
    pauli = [3, 3, 0]

    def tensors(gates, lc):
        return qtn.Network(3, gates, qtn.TN_EXPECTATION, pauli, lightcone=lc).wires()[1]

    assert tensors(tp, True) < tensors(tp, False)
    assert tensors(tp, True) == tensors(base, True)
    assert tensors(ntp, True) == tensors(ntp, False)
    two = base + [noise.channel_gate([np.kron(E, F) for E in noise.dephasing(0.2) for F in noise.dephasing(0.1)], 1, 2)]
    # the two-qubit channel touches qubit 1 (in the cone), so it stays and pulls qubit 2's past in
    assert tensors(two, True) == tensors(two, False) == tensors(base, True) + 4
    with pytest.raises(qtn.QtnError) as ei:
        qtn.Network(3, tp, qtn.TN_AMPLITUDE, [0, 0, 0])
    assert ei.value.code == qtn.TN_EINVAL
    with pytest.raises(qtn.QtnError):
        qtn.Network(3, base + [("SUPER1", 1, -1, -1, 0.0)], qtn.TN_EXPECTATION, pauli)


def _fold(kraus):
    """The documented folded layout, restated here: for Kraus operators E_k,
    entry (2a+b, 2c+d) is sum_k E_k[a, c] conj(E_k[b, d]); two-qubit entries
    are indexed (q0 out, q1 out, q0 in, q1 in), each wire value 2*ket + bra."""
    d = kraus[0].shape[0]
    q = 1 if d == 2 else 2
    S = np.zeros((4 ** q, 4 ** q), dtype=complex)
    for E in kraus:
        for a, b, c, dd in itertools.product(range(d), repeat=4):
            row = col = 0
            for j in range(q):
                sh = q - 1 - j
                row = row * 4 + 2 * ((a >> sh) & 1) + ((b >> sh) & 1)
                col = col * 4 + 2 * ((c >> sh) & 1) + ((dd >> sh) & 1)
            S[row, col] += E[a, c] * np.conj(E[b, dd])
    return S


def test_kraus_gates_fold_like_superoperators(qtn):
    """Channels given by Kraus operators (folded by tn_build) build the same
    networks as their superoperators in the documented layout: the same
    tensors and wires, the same light-cone decisions (trace preserving or
    not); malformed Kraus gates are refused."""
    from paper_1709_03636_amd import noise
    rng = np.random.default_rng(1)
    base = [("H", 0, -1, -1, 0.0), ("CNOT", 0, 1, -1, 0.0), ("H", 2, -1, -1, 0.0), ("CZ", 1, 2, -1, 0.0)]
    chans = [(noise.depolarizing(0.2), 2, -1), ([np.diag([1.0, 0.0])], 2, -1),
             ([np.kron(E, F) for E in noise.dephasing(0.2) for F in noise.amplitude_damping(0.3)], 1, 2),
             ([rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))], 0, 1)]
    for kraus, q0, q1 in chans:
        ks = [np.asarray(k, dtype=complex) for k in kraus]
        gk = base + [noise.channel_gate(ks, q0, q1)]
        gs = base + [("SUPER1" if q1 < 0 else "SUPER2", q0, q1, -1, 0.0, _fold(ks))]
        for lc in (True, False):
            nk = qtn.Network(3, gk, qtn.TN_EXPECTATION, [3, 3, 1], lightcone=lc)
            ns = qtn.Network(3, gs, qtn.TN_EXPECTATION, [3, 3, 1], lightcone=lc)
            wk, ws = nk.wires(), ns.wires()
            assert wk[:2] == ws[:2] and np.array_equal(wk[2], ws[2])
    for bad in (("KRAUS1", 0, -1, -1, 0.0, np.zeros((0, 2, 2))), ("KRAUS1", 0, -1, -1, 0.0)):
        with pytest.raises(qtn.QtnError) as ei:
            qtn.Network(3, base + [bad], qtn.TN_EXPECTATION, [3, 3, 1])
        assert ei.value.code == qtn.TN_EINVAL


@pytest.mark.parametrize("noisy", [False, True])
def test_qaoa_edge_lightcone_circuits_are_exact(qaoa, noisy):
    """The relabelled light-cone circuit of every edge gives the same <Z_u Z_v>
    as the whole circuit (density-matrix oracle), with and without a channel
    after every gate (which stops the ZZ layer from commuting as a block)."""
    from oracle import density, gates as og, statevector
    from paper_1709_03636_amd import noise
    n = 8
    e = workloads.random_regular_graph(3, n, 2)
    K = noise.depolarizing(0.05) if noisy else None
    p = 2
    ang = [0.37, -0.2, -0.61, 0.45]

    def ops_of(gl):
        ops = []
        for g in gl:
            kind, q0, q1, prm = g[0], g[1], g[2], g[3]
            if kind == "ZZ":
                ops.append(([og.zz(2 * ang[prm])], [q0, q1]))
            elif kind == "RX":
                ops.append(([og.rot(og.X, 2 * ang[prm])], [q0]))
            else:
                ops.append((K, [q0]))
        return ops

    def plus(m):
        return density.pure(statevector.product_state([[2 ** -0.5, 2 ** -0.5]] * m))

    rho = density.run(n, ops_of(qaoa.qaoa_gates(n, e, p, K)), plus(n))
    for u, v in e:
        full = density.expect_pauli(rho, [3 if q in (u, v) else 0 for q in range(n)]).real
        m, g = qaoa.edge_lightcone_circuit(n, e, p, (u, v), K)
        lc = density.expect_pauli(density.run(m, ops_of(g), plus(m)), [3, 3] + [0] * (m - 2)).real
        assert abs(full - lc) < 1e-13


def test_diagonal_mode_hyperedges_and_orders(qtn, qaoa):
    """Diagonal gates keep their wires: fewer wires, some held by more than
    two tensors; both order schemes return permutations, plans compile
    (forward and adjoint) and need fewer flops than the dense network."""
    e = workloads.random_regular_graph(3, 16, 1)
    dense = qaoa.edge_network(16, e, 2, e[0])
    diag = qaoa.edge_network(16, e, 2, e[0], diagonal=True)
    nw_d, nt_d, _ = dense.wires()
    nw, nt, ends = diag.wires()
    assert nt == nt_d and nw < nw_d
    for net in (dense, diag):
        for pi in (net.order_stochastic(3), net.order_linegraph(trials=3, seed=3)):
            assert sorted(pi.tolist()) == list(range(net.n_wires))
    dense.set_order(dense.order_linegraph(trials=4, seed=0))
    diag.set_order(diag.order_linegraph(trials=4, seed=0))
    a, b = dense.plan_info(), diag.plan_info()
    assert b["flops"] < a["flops"] / 4 and b["peak_bits"] <= a["peak_bits"]
    # ZZ leaves are 16-entry diagonals on existing wires: every wire of a ZZ leaf
    # also belongs to at least two other tensors
    steps = diag.plan_steps()
    assert len(steps) == b["n_steps"]


def test_state_vector_comparator_arguments(qtn):
    """Workspace size and argument checks of the state-vector comparator
    (all rejected before any device work)."""
    import ctypes
    import numpy as np
    L = qtn.lib()
    assert L.tn_sv_workspace_bytes(0) == -1 and L.tn_sv_workspace_bytes(35) == -1
    # 2^30 amplitudes of 8 bytes, then one FP64 partial sum per workgroup of the last pass (+1)
    assert L.tn_sv_workspace_bytes(30) == 8 * 2 ** 30 + 8 * (2 ** 25 // 256 + 1)
    assert L.tn_sv_workspace_bytes(3) == 8 * 8 + 8 * 2
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its checks first

    def call(n, edges, ws_bytes):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
        return L.tn_sv_maxcut_p1(n, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(e) // 2, 0.3, 0.2,
                                 fake, ws_bytes, fake, None)

    big = 1 << 40
    assert call(35, [(0, 1)], big) == qtn.TN_EINVAL
    assert call(8, [(3, 3)], big) == qtn.TN_EINVAL
    assert call(8, [(0, 8)], big) == qtn.TN_EINVAL
    assert call(8, [(0, 1)] * 257, big) == qtn.TN_EINVAL
    assert call(8, [(0, 1)], L.tn_sv_workspace_bytes(8) - 1) == qtn.TN_EINVAL


def test_binding_constants_match_header(qtn):
    """Every enumerator of the header has the same value in the binding."""
    hdr = open(os.path.join(ROOT, "include", "qtn.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    found = 0
    for body in re.findall(r"enum\s*\{(.*?)\}", hdr, re.S):
        value = -1
        for item in filter(None, (x.strip() for x in body.split(","))):
            name, _, expr = item.partition("=")
            name = name.strip()
            value = int(expr.strip(), 0) if expr.strip() else value + 1
            if hasattr(qtn, name):
                assert getattr(qtn, name) == value, name
                found += 1
    assert found >= 20
