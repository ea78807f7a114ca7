"""Host-side planning of every batching-grid batch through the library named
by QTN_LIB (a sanitizer build): seeded 4- and 5-regular graphs, n in
{50, 70, 100}, p in {1, 2}, 64 angle sets; networks built and ordered on 16
host threads (128 line-graph restarts per network at p = 2, as the benchmark
plans them), then batch planning in both matrix-core precisions. Also the
3-regular n=100 and n=60 batches, diagonal-gate networks and a gradient program
with recomputed forward runs under a memory limit. Prints one line
per batch; exits non-zero on any library error. Arguments "d,n,p" pick a
subset of the cases.

    python tests/sanitize/plan_grid.py [5,50,2 ...]"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from paper_1709_03636_amd import qaoa, qtn  # noqa: E402

cases = [(d, n, p) for d in (4, 5) for n in (50, 70, 100) for p in (1, 2)] + [(3, 100, 1), (3, 60, 2)]
if len(sys.argv) > 1:  # a subset: "d,n,p" arguments
    cases = [tuple(int(x) for x in a.split(",")) for a in sys.argv[1:]]
for d, n, p in cases:
    e = workloads.random_regular_graph(d, n, 0)
    for diagonal in (False, True):
        nets = qaoa.edge_networks(n, e, p, qtn.TN_C64, order="linegraph", trials=128 if p == 2 else 4,
                                  diagonal=diagonal, workers=16)
        b = qtn.Batch(nets, coef=[-0.5] * len(e), offset=0.5 * len(e), max_sets=64)
        b.set_precision(qtn.TN_MFMA_BF16X3)
        b.set_precision(qtn.TN_MFMA_FP32)
        info = b.info()
        print(d, n, p, "diagonal" if diagonal else "dense", info["n_fused"], info["n_global"], info["n_level"],
              b.workspace_bytes(), flush=True)
        del b, nets
# the adjoint program with forward runs recomputed under a memory limit
e = workloads.random_regular_graph(4, 10, 0)
full = qaoa.edge_network(10, e, 2, e[0], dtype=qtn.TN_C64, lightcone=False)
pi = full.order_linegraph(trials=8, seed=0)
full.set_order(pi)
cut = qaoa.edge_network(10, e, 2, e[0], dtype=qtn.TN_C64, lightcone=False)
cut.set_memory_limit(int(full.plan_info()["grad_bytes"] * 0.8))
cut.set_order(pi)
b = qtn.Batch([cut], max_sets=4)
b.set_precision(qtn.TN_MFMA_BF16X3)
print("recompute runs", cut.plan_info()["recompute_runs"], b.workspace_bytes(), flush=True)
print("ok")
