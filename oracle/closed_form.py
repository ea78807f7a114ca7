"""p=1 QAOA edge expectation in closed form (test infrastructure).

State: |psi> = exp(-i beta sum_q X_q) exp(-i gamma sum_E Z_i Z_j) |+>^n (the
QAOA circuit of Sec. QAOA / Max-Cut with p = 1). In the Heisenberg picture
Z_u Z_v becomes (c Z_u + s Y_u)(c Z_v + s Y_v) with c = cos 2beta,
s = sin 2beta. On |+>^n under the ZZ phases, <Z_u Z_v> = 0 and
  <Y_u Z_v> = sin 2gamma cos^{d_u - 1} 2gamma,
  <Y_u Y_v> = (1/2) cos^{d_u + d_v - 2 - 2 l} 2gamma (1 - cos^l 4gamma),
where d_u, d_v are the degrees and l the number of triangles through (u, v)
(common neighbours). Summing the four terms:
  <Z_u Z_v> = (1/2) sin 4beta sin 2gamma (cos^{d_u-1} 2gamma + cos^{d_v-1} 2gamma)
            + (1/2) sin^2 2beta cos^{d_u+d_v-2-2l} 2gamma (1 - cos^l 4gamma).
For a triangle-free d-regular graph this is sin 4beta sin 2gamma cos^{d-1} 2gamma.
"""
import numpy as np


def _graph_facts(n, edges):
    nb = [set() for _ in range(n)]
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return nb


def zz_p1(n, edges, gamma, beta):
    """<Z_u Z_v> for every edge at p = 1."""
    nb = _graph_facts(n, edges)
    c2g, s2g, c4g = np.cos(2 * gamma), np.sin(2 * gamma), np.cos(4 * gamma)
    s4b, s2b = np.sin(4 * beta), np.sin(2 * beta)
    out = []
    for u, v in edges:
        du, dv, lam = len(nb[u]), len(nb[v]), len(nb[u] & nb[v])
        t1 = 0.5 * s4b * s2g * (c2g ** (du - 1) + c2g ** (dv - 1))
        t2 = 0.5 * s2b ** 2 * c2g ** (du + dv - 2 - 2 * lam) * (1 - c4g ** lam)
        out.append(t1 + t2)
    return np.array(out)


def zz_p1_grad(n, edges, gamma, beta):
    """(d<ZZ>/dgamma, d<ZZ>/dbeta) per edge, by differentiating zz_p1 by hand."""
    nb = _graph_facts(n, edges)
    c2g, s2g = np.cos(2 * gamma), np.sin(2 * gamma)
    c4g, s4g = np.cos(4 * gamma), np.sin(4 * gamma)
    s4b, c4b, s2b, c2b = np.sin(4 * beta), np.cos(4 * beta), np.sin(2 * beta), np.cos(2 * beta)
    dg, db = [], []
    for u, v in edges:
        du, dv, lam = len(nb[u]), len(nb[v]), len(nb[u] & nb[v])

        def pw(e):  # d/dgamma cos^e(2 gamma)
            return 0.0 if e == 0 else -2.0 * e * c2g ** (e - 1) * s2g

        A = c2g ** (du - 1) + c2g ** (dv - 1)
        dA = pw(du - 1) + pw(dv - 1)
        e = du + dv - 2 - 2 * lam
        Bf = c2g ** e * (1 - c4g ** lam)
        dB = pw(e) * (1 - c4g ** lam) + c2g ** e * (4.0 * lam * c4g ** (lam - 1) * s4g if lam else 0.0)
        dg.append(0.5 * s4b * (2 * c2g * A + s2g * dA) + 0.5 * s2b ** 2 * dB)
        db.append(0.5 * 4 * c4b * s2g * A + 0.5 * 2 * s2b * 2 * c2b * Bf)
    return np.array(dg), np.array(db)


def cost_p1(n, edges, gamma, beta):
    """<C> = sum_E (1 - <Z_u Z_v>)/2 at p = 1."""
    return float(np.sum((1 - zz_p1(n, edges, gamma, beta)) / 2))
