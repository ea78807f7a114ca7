"""Test helpers: turn one seeded circuit description into both sides' inputs.

The circuit descriptions come from workloads (inputs only). The product side
receives gate tuples with parameter indices; the oracle side receives the
same gates with the angle already multiplied out. No arithmetic of the
method lives here.
"""
import numpy as np

import workloads

KIND_1Q_PARAM = {"RX", "RY", "RZ"}


def random_param_circuit(n, n_gates, seed, n_params=3):
    """(product gates, oracle gate list factory, params) for a seeded circuit.

    Rotations get a parameter index (coeff drawn from the description's
    angle); custom U1/U2 gates carry explicit matrices.
    """
    desc = workloads.random_circuit(n, n_gates, seed)
    rng = workloads.SplitMix64(seed + 77)
    params = [2.0 * rng.uniform() - 1.0 for _ in range(n_params)]
    prod, spec = [], []
    for kind, q0, q1, theta, mseed in desc:
        mat = None
        if kind == "U1":
            mat = np.array(workloads.random_unitary(2, mseed))
        elif kind == "U2":
            mat = np.array(workloads.random_unitary(4, mseed))
        if kind in KIND_1Q_PARAM or kind == "ZZ":
            p = rng.below(n_params + 1) - 1  # -1 = fixed angle
            coeff = theta if p < 0 else theta / 3.0
            prod.append((kind, q0, q1, p, coeff, mat))
            spec.append((kind, q0, q1, p, coeff, mseed))
        else:
            prod.append((kind, q0, q1, -1, 0.0, mat))
            spec.append((kind, q0, q1, -1, 0.0, mseed))

    def oracle_gates(prm):
        out = []
        for kind, q0, q1, p, coeff, mseed in spec:
            theta = coeff if p < 0 else coeff * prm[p]
            out.append((kind, q0, q1, theta, mseed))
        return out

    return prod, oracle_gates, np.array(params)


def gate_tuples_for_oracle(prod_gates, params):
    """Oracle gate tuples for product gates without custom matrices."""
    out = []
    for g in prod_gates:
        kind, q0, q1, p, coeff = g[:5]
        out.append((kind, q0, q1, coeff if p < 0 else coeff * params[p]))
    return out
