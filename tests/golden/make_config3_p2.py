"""Write tests/golden/config3_p2.json: FP64 oracle values for the p=2 batching
configuration (seeded random 4- and 5-regular graphs, n in {50, 70, 100}, 64
seeded angle sets), where no closed form exists and the light cones (17-42
qubits) are too wide for state vectors.

For each graph: <Z_u Z_v> on 64 sampled (edge, angle set) pairs by the
oracle's plain tensor-network contraction of the edge's light cone, and
d<Z_u Z_v>/d(gamma_1, gamma_2, beta_1, beta_2) on 4 of those pairs by the
parameter-shift rule on the same contraction. Calls only oracle/ and the
seeded input generators in workloads/.

    python tests/golden/make_config3_p2.py   (a few minutes on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import gates, gradients, tensornet  # noqa: E402

GRAPHS = [(4, 50), (4, 70), (4, 100), (5, 50), (5, 70), (5, 100)]
P, N_SETS, N_VALUES, N_GRADS = 2, 64, 64, 4


def sample_pairs(d, n, n_edges):
    """Distinct (edge index, angle set) pairs from a seeded generator."""
    rng = workloads.SplitMix64(1000 * d + n + 7)
    out = []
    while len(out) < N_VALUES:
        pr = (rng.below(n_edges), rng.below(N_SETS))
        if pr not in out:
            out.append(pr)
    return out


def value(args):
    n, edges, ang, edge = args
    gl = gates.qaoa_gate_list(n, edges, ang[:P], ang[P:])[n:]
    pauli = [0] * n
    pauli[edge[0]] = pauli[edge[1]] = 3
    return tensornet.expectation(n, gl, pauli, init=[np.array([1.0, 1.0]) / np.sqrt(2.0)] * n, lightcone=True).real


def grad(args):
    n, edges, ang, edge = args
    return gradients.parameter_shift_edge_tn(n, edges, np.asarray(ang), edge).tolist()


def main():
    out = {"source": "oracle/tensornet.py (light-cone folded network, FP64 tensordot) and "
                     "oracle/gradients.py parameter_shift_edge_tn",
           "p": P, "n_sets": N_SETS, "graph_seed": 0, "angle_seed": 0, "graphs": []}
    jobs_v, jobs_g, meta = [], [], []
    for d, n in GRAPHS:
        e = workloads.random_regular_graph(d, n, 0)
        ang = np.array(workloads.qaoa_angles(0, N_SETS, P))
        pairs = sample_pairs(d, n, len(e))
        meta.append((d, n, pairs))
        jobs_v += [(n, e, ang[s], e[i]) for i, s in pairs]
        jobs_g += [(n, e, ang[s], e[i]) for i, s in pairs[:N_GRADS]]
    with mp.get_context("fork").Pool(os.cpu_count()) as pool:
        gv = pool.map_async(grad, jobs_g, chunksize=1)
        vals = pool.map(value, jobs_v, chunksize=1)
        grads = gv.get()
    for k, (d, n, pairs) in enumerate(meta):
        out["graphs"].append({
            "d": d, "n": n,
            "values": [[i, s, vals[k * N_VALUES + j]] for j, (i, s) in enumerate(pairs)],
            "grads": [[i, s, grads[k * N_GRADS + j]] for j, (i, s) in enumerate(pairs[:N_GRADS])]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_p2.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
