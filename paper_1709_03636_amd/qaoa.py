"""QAOA Max-Cut on top of the contraction library (Sec. QAOA / Max-Cut).

The circuit: |+>^n (the Hadamard layer folded into the initial product
state), then for k = 1..p the phase separator exp(-i gamma_k Z_u Z_v) on every
edge (TN_ZZ with theta = 2 gamma_k) and the mixer exp(-i beta_k X) on every
qubit (TN_RX with theta = 2 beta_k). Parameters are ordered
(gamma_1..gamma_p, beta_1..beta_p). The cost <C> = sum_E (1 - <Z_u Z_v>)/2 is
evaluated with one folded light-cone network per edge (measurement Z on u and
v, trace elsewhere), combined on the GPU in FP64.
"""
import math
import os

import numpy as np

from . import noise as noise_mod
from . import qtn

PLUS = [1 / math.sqrt(2), 0.0, 1 / math.sqrt(2), 0.0]


def _zz_layer(edges, k, chan):
    out = []
    for u, v in edges:
        out.append(("ZZ", u, v, k, 2.0))
        if chan is not None:
            out += [chan(u), chan(v)]
    return out


def _rx_layer(qubits, p, k, chan):
    out = []
    for q in qubits:
        out.append(("RX", q, -1, p + k, 2.0))
        if chan is not None:
            out.append(chan(q))
    return out


def _channel(noise):
    """noise: None or the Kraus operators of a one-qubit channel applied
    after every gate, on each qubit the gate acts on."""
    if noise is None:
        return None
    return lambda q: noise_mod.channel_gate(noise, q)


def qaoa_gates(n, edges, p, noise=None):
    """Gate tuples of the QAOA circuit without the Hadamard layer."""
    chan = _channel(noise)
    gates = []
    for k in range(p):
        gates += _zz_layer(edges, k, chan)
        gates += _rx_layer(range(n), p, k, chan)
    return gates


def _lightcone_in_sequence(n, edges, p, edge, noise):
    """With channels between the ZZ gates the ZZ layer no longer commutes as
    a block: walk the gate sequence backwards, keeping a gate when it touches
    the support (which then takes its qubits). Kept qubits are relabelled
    u -> 0, v -> 1, then in order of their last appearance."""
    full = qaoa_gates(n, edges, p, noise)
    sup = {edge[0], edge[1]}
    kept = []
    for g in reversed(full):
        qs = [g[1]] + ([g[2]] if g[2] >= 0 else [])
        if any(q in sup for q in qs):
            kept.append(g)
            sup.update(qs)
    kept.reverse()
    lab = {edge[0]: 0, edge[1]: 1}
    for g in reversed(kept):
        for q in (g[1], g[2]):
            if q >= 0 and q not in lab:
                lab[q] = len(lab)
    gates = []
    for g in kept:
        q0, q1 = lab[g[1]], (lab[g[2]] if g[2] >= 0 else -1)
        gates.append((g[0], q0, q1) + tuple(g[3:]))
    return len(lab), gates


def edge_lightcone_circuit(n, edges, p, edge, noise=None):
    """The gates that can reach <Z_u Z_v>, on the light-cone qubits only,
    relabelled canonically: u -> 0, v -> 1, then breadth-first over the kept
    ZZ gates with ties broken by already-assigned neighbour labels. Isomorphic
    light cones thus give identical circuits (hence identical contraction
    programs, which the batch stores once). Returns (m qubits, gates).
    With noise the cone follows the gate sequence instead (see
    _lightcone_in_sequence)."""
    if noise is not None:
        return _lightcone_in_sequence(n, edges, p, edge, noise)
    adj = {}
    for a, b in edges:
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    sup = {edge[0], edge[1]}
    layers = []
    for _ in range(p):  # backwards: a ZZ layer is kept where it touches the support
        zz = [(a, b) for (a, b) in edges if a in sup or b in sup]
        layers.append(zz)
        sup = sup | {q for e in zz for q in e}
    layers.reverse()
    kadj = {}
    for zz in layers:
        for a, b in zz:
            kadj.setdefault(a, set()).add(b)
            kadj.setdefault(b, set()).add(a)
    lab = {edge[0]: 0, edge[1]: 1}
    frontier = [edge[0], edge[1]]
    while frontier:
        cand = {w for q in frontier for w in kadj.get(q, ()) if w not in lab}
        cand = sorted(cand, key=lambda w: (sorted(lab[x] for x in kadj[w] if x in lab), len(kadj[w])))
        for w in cand:
            lab[w] = len(lab)
        frontier = cand
    m = len(lab)
    gates = []
    for k, zz in enumerate(layers):
        ren = sorted(tuple(sorted((lab[a], lab[b]))) for a, b in zz)
        gates += _zz_layer(ren, k, None)
        gates += _rx_layer(range(m), p, k, None)
    return m, gates


def edge_network(n, edges, p, edge, dtype=qtn.TN_C64, lightcone=True, noise=None, diagonal=False):
    """Folded network of <Z_u Z_v>. With lightcone=True it is built on the
    edge's canonically relabelled light-cone circuit; with lightcone=False it
    is the whole circuit (trace on every other qubit). noise: Kraus operators
    of a trace-preserving one-qubit channel after every gate (or None).
    diagonal: the ZZ gates become 16-entry tensors on hyperedge wires
    (tn_target.diagonal) instead of dense 256-entry superoperators."""
    if lightcone:
        m, gates = edge_lightcone_circuit(n, edges, p, edge, noise)
        pauli = [3, 3] + [0] * (m - 2)
    else:
        m, gates = n, qaoa_gates(n, edges, p, noise)
        pauli = [0] * n
        pauli[edge[0]] = pauli[edge[1]] = 3
    init = np.array([complex(PLUS[0], PLUS[1]), complex(PLUS[2], PLUS[3])] * m)
    return qtn.Network(m, gates, qtn.TN_EXPECTATION, pauli, n_params=2 * p, init=init, dtype=dtype,
                       lightcone=lightcone, diagonal=diagonal)


def edge_networks(n, edges, p, dtype=qtn.TN_C64, order="stochastic", seed=0, trials=8, lightcone=True, noise=None,
                  diagonal=False, workers=None):
    """One network per edge with its contraction order set. The networks are
    built and ordered on `workers` host threads (default: up to 16; the
    library's host calls release the interpreter lock and share no state);
    each order depends only on its network and seed."""
    if order not in ("stochastic", "linegraph"):
        raise ValueError(order)

    def one(e):
        net = edge_network(n, edges, p, e, dtype, lightcone, noise, diagonal)
        pi = net.order_stochastic(seed) if order == "stochastic" else net.order_linegraph(trials=trials, seed=seed)
        net.set_order(pi)
        return net

    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or len(edges) < 8:
        return [one(e) for e in edges]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, edges))


class MaxCut:
    """<C>(params) and its gradient for many parameter vectors at once."""

    def __init__(self, n, edges, p, dtype=qtn.TN_C64, order="stochastic", seed=0, max_sets=64, trials=8, noise=None,
                 diagonal=False):
        self.n, self.edges, self.p = n, list(edges), p
        self.nets = edge_networks(n, edges, p, dtype, order, seed, trials, noise=noise, diagonal=diagonal)
        m = len(self.edges)
        self.batch = qtn.Batch(self.nets, coef=[-0.5] * m, offset=0.5 * m, max_sets=max_sets)

    def expectation(self, params, out=None):
        import torch
        params = torch.as_tensor(params, dtype=torch.float64, device="cuda").reshape(-1, 2 * self.p).contiguous()
        obj = torch.empty(params.shape[0], dtype=torch.float64, device="cuda")
        self.batch.contract(params, out=out, obj=obj)
        return obj

    def value_and_grad(self, params, out=None):
        import torch
        params = torch.as_tensor(params, dtype=torch.float64, device="cuda").reshape(-1, 2 * self.p).contiguous()
        obj = torch.empty(params.shape[0], dtype=torch.float64, device="cuda")
        grad = torch.empty_like(params)
        self.batch.grad(params, out=out, obj=obj, grad=grad)
        return obj, grad


def make_autograd():
    import torch

    class QAOAExpectation(torch.autograd.Function):
        """<C>(params) with the adjoint-contraction gradient as its backward."""

        @staticmethod
        def forward(ctx, params, model):
            obj, grad = model.value_and_grad(params.detach())
            ctx.save_for_backward(grad)
            return obj

        @staticmethod
        def backward(ctx, gobj):
            (grad,) = ctx.saved_tensors
            return gobj.reshape(-1, 1) * grad, None

    return QAOAExpectation
