"""Write tests/golden/bench_refs.json: the FP64 oracle values bench.py checks
its GPU results against (bench.py itself runs the oracle only for its CPU
baseline). Seeded inputs from workloads/ (graph seed 0, angle seed 0, 64
angle sets), the same as bench.py's. Calls only oracle/ and workloads/.

  * 3-regular n=100 p=1 (the plain and batched p=1 rows): <C> and
    d<C>/d(gamma, beta) of every angle set; <Z_u Z_v> and its derivative on
    every edge for sets 0, 21, 42 and 63 (p=1 closed form, exact);
  * 4- and 5-regular n in {50, 70, 100}, p=1 (batching grid): <Z_u Z_v> on
    every edge for sets 0, 21, 42 and 63 (closed form);
  * 3-regular n=60 p=2 (differentiation row): <C> of sets 0, 16, 32 and 48
    by light-cone state vectors, d<C>/d(params) of set 1 by the
    parameter-shift rule on the light cones;
  * whole-circuit networks of edge 0 (dense-regime and diagonal rows):
    6-regular n=20 and n=30, set 0, closed form;
  * crossover rows: <C> at gamma=0.4, beta=0.3 for d-regular graphs, d = 3..7,
    n in {30, 40}, and <Z_u Z_v> of edge 0 at n=30 (closed form).

    python tests/golden/make_bench_refs.py   (about a minute on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import closed_form, gradients, statevector  # noqa: E402

N_SETS, SAMPLE_SETS = 64, (0, 21, 42, 63)


def p1_block(d, n, full):
    e = workloads.random_regular_graph(d, n, 0)
    ang = np.array(workloads.qaoa_angles(0, N_SETS, 1))
    out = {"d": d, "n": n, "p": 1, "sets": list(SAMPLE_SETS), "zz": [], "dzz": []}
    for s in SAMPLE_SETS:
        out["zz"].append(closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1]).tolist())
        dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
        out["dzz"].append(np.stack([dg, db], axis=1).tolist())
    if full:
        out["cost"], out["grad"] = [], []
        for s in range(N_SETS):
            out["cost"].append(closed_form.cost_p1(n, e, ang[s, 0], ang[s, 1]))
            dg, db = closed_form.zz_p1_grad(n, e, ang[s, 0], ang[s, 1])
            out["grad"].append([-0.5 * float(dg.sum()), -0.5 * float(db.sum())])
    return out


def _sv_edge(args):
    n, e, a, p, ed = args
    return statevector.qaoa_zz_edge(n, e, a[:p], a[p:], ed)


def _ps_edge(args):
    n, e, a, ed = args
    return gradients.parameter_shift_edge(n, e, a, ed)


def main():
    refs = {"source": "oracle/closed_form.py, oracle/statevector.py, oracle/gradients.py", "graph_seed": 0,
            "angle_seed": 0, "n_sets": N_SETS}
    refs["d3_n100_p1"] = p1_block(3, 100, True)
    refs["grid_p1"] = [p1_block(d, n, False) for d in (4, 5) for n in (50, 70, 100)]
    # differentiation row: 3-regular n=60, p=2
    n, p = 60, 2
    e = workloads.random_regular_graph(3, n, 0)
    ang = np.array(workloads.qaoa_angles(0, N_SETS, p))
    with mp.get_context("fork").Pool(os.cpu_count()) as pool:
        cost = {}
        for s in (0, 16, 32, 48):
            zz = pool.map(_sv_edge, [(n, e, ang[s], p, ed) for ed in e])
            cost[s] = float(np.sum((1 - np.array(zz)) / 2))
        ps = pool.map(_ps_edge, [(n, e, ang[1], ed) for ed in e])
    refs["d3_n60_p2"] = {"cost_sets": sorted(cost), "cost": [cost[s] for s in sorted(cost)], "grad_set": 1,
                         "grad": (-0.5 * np.sum(ps, axis=0)).tolist()}
    # whole-circuit networks of edge 0, set 0, p=1
    a0 = np.array(workloads.qaoa_angles(0, N_SETS, 1))[0]
    whole = {}
    for d, n in ((6, 20), (6, 30)):
        e = workloads.random_regular_graph(d, n, 0)
        dg, db = closed_form.zz_p1_grad(n, e, a0[0], a0[1])
        whole[f"d{d}_n{n}"] = {"zz_edge0": float(closed_form.zz_p1(n, e, a0[0], a0[1])[0]),
                               "dzz_edge0": [float(dg[0]), float(db[0])]}
    refs["whole_circuit_edge0_set0"] = whole
    # crossover rows
    cross = []
    for n in (30, 40):
        for d in (3, 4, 5, 6, 7):
            e = workloads.random_regular_graph(d, n, 0)
            cross.append({"d": d, "n": n, "cost": closed_form.cost_p1(n, e, 0.4, 0.3),
                          "zz_edge0": float(closed_form.zz_p1(n, e, 0.4, 0.3)[0])})
    refs["crossover_g0.4_b0.3"] = cross
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_refs.json")
    with open(path, "w") as f:
        json.dump(refs, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
