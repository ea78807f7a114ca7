"""The stored oracle values bench.py checks against (tests/golden/bench_refs.json,
written by tests/golden/make_bench_refs.py from oracle/ only) agree with the
oracle recomputed here on a sample, and bench.py refuses more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np

import workloads
from oracle import closed_form

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REFS = json.load(open(os.path.join(ROOT, "tests", "golden", "bench_refs.json")))


def test_p1_blocks_match_closed_form():
    ang = np.array(workloads.qaoa_angles(0, 64, 1))
    for blk in [REFS["d3_n100_p1"]] + REFS["grid_p1"][::2]:
        e = workloads.random_regular_graph(blk["d"], blk["n"], 0)
        j = 1
        s = blk["sets"][j]
        assert np.allclose(blk["zz"][j], closed_form.zz_p1(blk["n"], e, ang[s, 0], ang[s, 1]), atol=1e-14)
    blk = REFS["d3_n100_p1"]
    e = workloads.random_regular_graph(3, 100, 0)
    # objective and gradient of a set against the per-edge values they combine
    j, s = 2, blk["sets"][2]
    assert abs(blk["cost"][s] - np.sum((1 - np.array(blk["zz"][j])) / 2)) < 1e-12
    assert np.allclose(blk["grad"][s], -0.5 * np.array(blk["dzz"][j]).sum(axis=0), atol=1e-12)
    assert abs(blk["cost"][5] - closed_form.cost_p1(100, e, ang[5, 0], ang[5, 1])) < 1e-12


def test_crossover_and_whole_circuit_values():
    for r in REFS["crossover_g0.4_b0.3"][::3]:
        e = workloads.random_regular_graph(r["d"], r["n"], 0)
        assert abs(r["cost"] - closed_form.cost_p1(r["n"], e, 0.4, 0.3)) < 1e-12
    a0 = np.array(workloads.qaoa_angles(0, 64, 1))[0]
    e = workloads.random_regular_graph(6, 20, 0)
    assert abs(REFS["whole_circuit_edge0_set0"]["d6_n20"]["zz_edge0"] - closed_form.zz_p1(20, e, *a0)[0]) < 1e-14


def test_differentiation_refs_are_consistent():
    r = REFS["d3_n60_p2"]
    assert r["cost_sets"] == [0, 16, 32, 48] and len(r["grad"]) == 4
    # <C> of a 90-edge graph lies in [0, 90]; the expected cut at these angles is well inside
    assert all(0.0 < c < 90.0 for c in r["cost"])


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout
