"""Answer-string estimation (Sec. "Estimating the answer string").

Qubit by qubit: one closed-network contraction gives the probability that
the qubits fixed so far read their chosen values and the current qubit reads
0 (projectors on those qubits, trace on the rest); the probability of reading
1 is what remains of the prefix probability. The likelier value is kept
(a random choice when both are equally likely, up to a stated relative
tolerance) and becomes a projector in the next contraction: n contractions
for n qubits, each on the GPU through the plain one-network path.
"""
import numpy as np

from . import qtn


def answer_string(n, gates, init=None, n_params=0, params=(), dtype=qtn.TN_C128, tie_tol=1e-9,
                  tie_draws=None, order="linegraph", trials=4, seed=0, lightcone=True):
    """Returns (bits, probs): the chosen bit of every qubit (qubit 0 first)
    and, per qubit, the pair (P(prefix, 0), P(prefix, 1)).

    tie_tol: the two outcomes count as equally likely when they differ by at
    most tie_tol times the prefix probability; tie_draws[k] (0 or 1) is then
    the choice for qubit k (the random draw, passed in so the result is
    reproducible; default all zeros)."""
    draws = np.zeros(n, dtype=np.int64) if tie_draws is None else np.asarray(tie_draws)
    bits, probs = [], []
    p_prefix = 1.0
    for k in range(n):
        target = [bits[q] if q < k else (0 if q == k else 2) for q in range(n)]
        net = qtn.Network(n, gates, qtn.TN_PROBABILITY, target, n_params=n_params, init=init, dtype=dtype,
                          lightcone=lightcone)
        if order == "linegraph":
            net.set_order(net.order_linegraph(trials=trials, seed=seed))
        else:
            net.set_order(net.order_stochastic(seed))
        p0 = net.contract(params).real
        p1 = p_prefix - p0
        if abs(p0 - p1) <= tie_tol * p_prefix:
            b = int(draws[k])
        else:
            b = 0 if p0 > p1 else 1
        probs.append((p0, p1))
        bits.append(b)
        p_prefix = p0 if b == 0 else p1
    return bits, probs


def cut_value(edges, bits):
    """Number of edges whose endpoints read different bits."""
    return sum(1 for u, v in edges if bits[u] != bits[v])
