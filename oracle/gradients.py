"""Gradients of QAOA <C> for the oracle (test infrastructure).

Two routes:
  * central finite differences, (f(x+h) - f(x-h)) / 2h in FP64; its
    truncation error is O(h^2) times the third derivative;
  * the parameter-shift rule: for a gate exp(-i theta G) with G^2 = I,
    d/dtheta <O> = <O>(theta + pi/4) - <O>(theta - pi/4) exactly; a QAOA angle
    enters every ZZ phase (gamma_k) or every X rotation (beta_k) of its layer,
    so its derivative is the sum of the shifts of each occurrence.
Both evaluate <C> by brute-force state vectors (statevector.run).
"""
import numpy as np

from . import gates, statevector


def _cost_from_gates(n, edges, gl):
    prob = np.abs(statevector.run(n, gl)) ** 2
    sign = np.array([1.0, -1.0])
    tot = 0.0
    for (u, v) in edges:
        marg = np.moveaxis(prob, [u, v], [0, 1]).reshape(2, 2, -1).sum(axis=2)
        tot += (1.0 - sign @ marg @ sign) / 2.0
    return float(tot)


def cost(n, edges, params):
    """<C> for params = (gamma_1..gamma_p, beta_1..beta_p)."""
    p = len(params) // 2
    return _cost_from_gates(n, edges, gates.qaoa_gate_list(n, edges, params[:p], params[p:]))


def finite_difference(n, edges, params, h=1e-4):
    params = np.asarray(params, dtype=np.float64)
    g = np.zeros_like(params)
    for i in range(len(params)):
        e = np.zeros_like(params)
        e[i] = h
        g[i] = (cost(n, edges, params + e) - cost(n, edges, params - e)) / (2 * h)
    return g


def parameter_shift(n, edges, params):
    """d<C>/d(gamma_k, beta_k) by shifting every gate occurrence by +-pi/4.

    A gate exp(-i a G) appears in the gate list as ZZ(2a) or R_X(2a), so a
    shift of a by pi/4 is a shift of the listed angle by pi/2.
    """
    p = len(params) // 2
    base = gates.qaoa_gate_list(n, edges, params[:p], params[p:])
    g = np.zeros(2 * p)
    # layer k of the gate list: n H gates, then per layer |E| ZZ and n RX
    per_layer = len(edges) + n
    for k in range(p):
        start = n + k * per_layer
        for idx in range(start, start + per_layer):
            kind = base[idx][0]
            slot = k if kind == "ZZ" else p + k
            plus = list(base)
            minus = list(base)
            kd, q0, q1, th = base[idx]
            plus[idx] = (kd, q0, q1, th + np.pi / 2)
            minus[idx] = (kd, q0, q1, th - np.pi / 2)
            g[slot] += _cost_from_gates(n, edges, plus) - _cost_from_gates(n, edges, minus)
    return g


def parameter_shift_edge(n, edges, params, edge):
    """d<Z_u Z_v>/d(gamma_k, beta_k) for one edge, by the shift rule on the
    edge's light-cone circuit (state vector over the light cone only)."""
    p = len(params) // 2
    m, sub, uv, pos = statevector.qaoa_edge_lightcone_circuit(n, edges, params[:p], params[p:], edge,
                                                              with_index=True)
    per_layer = len(edges) + n
    g = np.zeros(2 * p)
    for idx, ((kd, q0, q1, th), full) in enumerate(zip(sub, pos)):
        if kd == "H":
            continue
        k = (full - n) // per_layer
        slot = k if kd == "ZZ" else p + k
        plus, minus = list(sub), list(sub)
        plus[idx] = (kd, q0, q1, th + np.pi / 2)
        minus[idx] = (kd, q0, q1, th - np.pi / 2)
        g[slot] += statevector.zz_of(m, plus, uv) - statevector.zz_of(m, minus, uv)
    return g


def parameter_shift_edge_tn(n, edges, params, edge):
    """d<Z_u Z_v>/d(gamma_k, beta_k) for one edge by the shift rule, each
    shifted circuit evaluated by the plain tensor-network contraction of its
    light cone (for light cones too wide for a state vector).

    The kept gates are found once on the tagged gate list (the light cone does
    not depend on the angles); every occurrence of an angle is shifted by
    +-pi/4 in turn (+-pi/2 in the listed ZZ(2a) or R_X(2a) angle) and the two
    folded networks are contracted.
    """
    from . import tensornet
    p = len(params) // 2
    gl = gates.qaoa_gate_list(n, edges, params[:p], params[p:])
    tagged = [g + (i,) for i, g in enumerate(gl)][n:]  # the H layer is the |+> boundary
    kept, sup = tensornet.light_cone(n, tagged, {edge[0], edge[1]})
    ops = [gates.PAULI[3] if q in edge else gates.PAULI[0] for q in range(n)]
    plus = [np.array([1.0, 1.0]) / np.sqrt(2.0)] * n
    per_layer = len(edges) + n

    def zz(gate_list):
        net = tensornet.folded_network(n, [g[:4] for g in gate_list], ops, init=plus, qubits=sup)
        return tensornet.contract(net).real

    g = np.zeros(2 * p)
    for idx, (kd, q0, q1, th, full) in enumerate(kept):
        k = (full - n) // per_layer
        slot = k if kd == "ZZ" else p + k
        plus_l, minus_l = list(kept), list(kept)
        plus_l[idx] = (kd, q0, q1, th + np.pi / 2, full)
        minus_l[idx] = (kd, q0, q1, th - np.pi / 2, full)
        g[slot] += zz(plus_l) - zz(minus_l)
    return g
