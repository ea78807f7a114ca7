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


def edge_network(n, edges, p, edge, dtype=qtn.TN_C64, lightcone=True):
    u, v = edge
    pauli = [0] * n
    pauli[u] = pauli[v] = 3
    init = np.array([complex(PLUS[0], PLUS[1]), complex(PLUS[2], PLUS[3])] * n)
    return qtn.Network(n, qaoa_gates(n, edges, p), qtn.TN_EXPECTATION, pauli, n_params=2 * p, init=init,
                       dtype=dtype, lightcone=lightcone)


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
