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

import numpy as np

from . import qtn

PLUS = [1 / math.sqrt(2), 0.0, 1 / math.sqrt(2), 0.0]


def qaoa_gates(n, edges, p):
    """Gate tuples of the QAOA circuit without the Hadamard layer."""
    gates = []
    for k in range(p):
        gates += [("ZZ", u, v, k, 2.0) for (u, v) in edges]
        gates += [("RX", q, -1, p + k, 2.0) for q in range(n)]
    return gates


def edge_lightcone_circuit(n, edges, p, edge):
    """The gates that can reach <Z_u Z_v>, on the light-cone qubits only,
    relabelled canonically: u -> 0, v -> 1, then breadth-first over the kept
    ZZ gates with ties broken by already-assigned neighbour labels. Isomorphic
    light cones thus give identical circuits (hence identical contraction
    programs, which the batch stores once). Returns (m qubits, gates)."""
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
        gates += [("ZZ", a, b, k, 2.0) for a, b in ren]
        gates += [("RX", q, -1, p + k, 2.0) for q in range(m)]
    return m, gates


def edge_network(n, edges, p, edge, dtype=qtn.TN_C64, lightcone=True):
    """Folded network of <Z_u Z_v>. With lightcone=True it is built on the
    edge's canonically relabelled light-cone circuit; with lightcone=False it
    is the whole circuit (trace on every other qubit)."""
    if lightcone:
        m, gates = edge_lightcone_circuit(n, edges, p, edge)
        pauli = [3, 3] + [0] * (m - 2)
    else:
        m, gates = n, qaoa_gates(n, edges, p)
        pauli = [0] * n
        pauli[edge[0]] = pauli[edge[1]] = 3
    init = np.array([complex(PLUS[0], PLUS[1]), complex(PLUS[2], PLUS[3])] * m)
    return qtn.Network(m, gates, qtn.TN_EXPECTATION, pauli, n_params=2 * p, init=init, dtype=dtype,
                       lightcone=lightcone)


def edge_networks(n, edges, p, dtype=qtn.TN_C64, order="stochastic", seed=0, trials=8, lightcone=True):
    """One network per edge with its contraction order set."""
    nets = []
    for e in edges:
        net = edge_network(n, edges, p, e, dtype, lightcone)
        if order == "stochastic":
            pi = net.order_stochastic(seed)
        elif order == "linegraph":
            pi = net.order_linegraph(trials=trials, seed=seed)
        else:
            raise ValueError(order)
        net.set_order(pi)
        nets.append(net)
    return nets


class MaxCut:
    """<C>(params) and its gradient for many parameter vectors at once."""

    def __init__(self, n, edges, p, dtype=qtn.TN_C64, order="stochastic", seed=0, max_sets=64, trials=8):
        self.n, self.edges, self.p = n, list(edges), p
        self.nets = edge_networks(n, edges, p, dtype, order, seed, trials)
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
