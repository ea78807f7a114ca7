"""Benchmark: batched QAOA <Z_u Z_v> network contraction, forward + adjoint gradient.

Headline workload (the largest batching configuration): QAOA p=2 Max-Cut on
a seeded random 5-regular graph with 100 vertices (250 edges), one folded
light-cone network per edge, line-graph (min-fill) contraction order (best
of 128 restarts), 64 angle sets (gamma_1, gamma_2, beta_1, beta_2) uniform
in [0, pi) from seed 0; complex64 contraction with split-BF16 matrix-core
products (FP32 accumulation), FP64 final scalars and gradient sums. One step
= one pass of the whole path over the batch: angle binding, every pairwise
contraction, the final scalars, the adjoint sweep and the objective and
gradient combine, replayed from a captured HIP graph.

After the timed steps, the last replay's per-network values and gradients
are checked against FP64 oracle values stored in tests/golden (written by
committed scripts that call only the oracle); a miss fails the run. Also
measured: forward-only throughput, each executor's kernel time and roofline
figures, the 3-regular n=100 p=1 batch (plain one-network-per-launch path in
complex64 and complex128, and batched), the dense regime on the matrix
cores, the rows past the hot path, the other batching configurations, the
differentiation and crossover rows, and the FP64 CPU oracle timed on a
bounded sample of the headline workload and of the p=1 batch.

Prints one JSON line (rank 0).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HEAD_D, HEAD_N, HEAD_P = 5, 100, 2
N_SETS, GRAPH_SEED, ANGLE_SEED = 64, 0, 0
# restarts of the line-graph order search per network: at p = 2 on 5-regular graphs the best of 128 has
# 2-4x fewer flops than the best of 4 (plan time, on host threads)
GRID_TRIALS = {1: 4, 2: 128}
HBM_PEAK = 8.0e12
FP32_MFMA_PEAK = 157.3e12
FP64_MFMA_PEAK = 78.6e12
BF16_MFMA_PEAK = 2.5e15
FP32_VALU_PEAK = 157.3e12  # published FP32 vector peak (packed FP32); 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# x 2.4 GHz = 78.6e12 without packed instructions, which this build does not emit
# split-BF16 tolerances (complex64 with three bf16 products per real product, FP32 accumulation):
# <Z_u Z_v> values and per-network gradients, absolute (derivation in the GPU configuration tests)
TOL_ZZ_BF16, TOL_G_BF16 = 5e-5, 5e-4
BOX_CORES = 16  # host cores the GPU machine allots to one GPU (worker pools stay within it)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_refs():
    """Oracle values for the checks (tests/golden, written by scripts that call only oracle/)."""
    g = os.path.join(ROOT, "tests", "golden")
    refs = json.load(open(os.path.join(g, "bench_refs.json")))
    refs["config3_p2"] = {(x["d"], x["n"]): x for x in json.load(open(os.path.join(g, "config3_p2.json")))["graphs"]}
    return refs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(args):
    """One (edge, angle set) network by the FP64 oracle: the value and the
    central finite-difference gradient in every parameter (1 + 4p plain
    tensordot contractions of the edge's light cone)."""
    n, edges, p, edge, params = args
    from threadpoolctl import threadpool_limits
    from oracle import tensornet, gates
    with threadpool_limits(1):
        def zz(prm):
            gl = gates.qaoa_gate_list(n, edges, prm[:p], prm[p:])[n:]
            plus = [np.array([1.0, 1.0]) / np.sqrt(2.0)] * n
            pauli = [0] * n
            pauli[edge[0]] = pauli[edge[1]] = 3
            return tensornet.expectation(n, gl, pauli, init=plus, lightcone=True).real
        v = zz(params)
        h = 1e-4
        g = []
        for i in range(2 * p):
            e = np.zeros(2 * p)
            e[i] = h
            g.append((zz(params + e) - zz(params - e)) / (2 * h))
    return v, g


def cpu_baseline(n, edges, p, angles, budget_s, label):
    """The FP64 oracle (plain tensordot contraction, forward plus
    finite-difference gradient per network) on a bounded sample of a batch's
    (edge, angle set) networks, in worker processes on the machine's cores."""
    import multiprocessing as mp
    workers = max(1, min(BOX_CORES, os.cpu_count() or 1))
    # sample: edges in a seeded order, angle sets round robin
    rng = np.random.default_rng(1234)
    order = rng.permutation(len(edges))
    tasks = [(n, edges, p, edges[int(order[k % len(edges)])], np.array(angles[k % angles.shape[0]]))
             for k in range(len(edges) * angles.shape[0])]
    t0 = time.perf_counter()
    _oracle_worker(tasks[0])
    one = time.perf_counter() - t0
    n_sample = int(min(len(tasks), max(workers, budget_s * workers / max(one, 1e-4))))
    sample = tasks[:n_sample]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_worker, sample, chunksize=1)
        dt = time.perf_counter() - t0
    # one core: a short sample in this process
    n1 = int(max(1, min(len(tasks), 3.0 / max(one, 1e-4))))
    t0 = time.perf_counter()
    for t in tasks[:n1]:
        _oracle_worker(t)
    dt1 = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "networks/s (fwd+grad)", "cores": workers, "kind": "oracle",
            "value_1core": n1 / dt1, "sample_1core": n1,
            "sample": f"{n_sample} of the {len(tasks)} (edge, angle set) networks of {label}, each forward plus "
                      f"central finite-difference gradient ({1 + 4 * p} FP64 light-cone contractions), "
                      f"{workers} worker processes with one BLAS thread each",
            "seconds": dt, "host_cpu": cpu_model(), "host_cpu_count": os.cpu_count(),
            "cores_note": f"the GPU box allots {BOX_CORES} host cores to one GPU; pools stay within them"}


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1709_03636_amd", "csrc"))):
        if f.endswith((".hip", ".hpp", ".cpp")):  # kernels and the planner that writes their programs
            h.update(open(os.path.join(ROOT, "paper_1709_03636_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(tag, kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary (profiles/traffic.<tag>.json), or None
    when the summary covers another kernel or the device sources changed
    since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic.{tag}.json")))
    except (OSError, ValueError):
        return None
    if rec.get("device_src_sha256_prefix") != kernel_src_sha() or rec.get("kernel") != kernel:
        return None
    return rec["traffic_bytes_per_launch"]


def copy_calibration(steps):
    """A plain device copy of known size, for scaling HBM traffic counters."""
    import torch
    n = 256 << 20
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    for _ in range(steps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": steps}))


def max_cut_brute_force(n, edges):
    """Exact Max-Cut by enumerating every cut with vertex n-1 on side 0."""
    x = np.arange(1 << (n - 1), dtype=np.int64)
    cut = np.zeros(x.shape, dtype=np.int64)
    for u, v in edges:
        cut += ((x >> u) ^ (x >> v)) & 1
    return int(cut.max())


def p1_errors(block, out, gnet=None, obj=None, grad=None):
    """Largest deviations of a p=1 batch's results from the stored closed-form
    values: per-edge <Z_u Z_v> (and gradients) on the sampled sets, the
    objective and its gradient on every set (when stored)."""
    o = out.cpu().numpy()
    r = {"max_abs_zz": max(float(np.max(np.abs(o[:, s, 0] - np.array(block["zz"][j]))))
                           for j, s in enumerate(block["sets"]))}
    if gnet is not None:
        g = gnet.cpu().numpy()
        r["max_abs_grad_net"] = max(float(np.max(np.abs(g[:, s, :] - np.array(block["dzz"][j]))))
                                    for j, s in enumerate(block["sets"]))
    if obj is not None and "cost" in block:
        c = np.array(block["cost"][:obj.shape[0]])
        r["max_rel_cost"] = float(np.max(np.abs(obj.cpu().numpy() - c) / np.maximum(1.0, np.abs(c))))
    if grad is not None and "grad" in block:
        gr = np.array(block["grad"][:grad.shape[0]])
        r["max_rel_grad"] = float(np.max(np.abs(grad.cpu().numpy() - gr)) / max(1.0, np.abs(gr).max()))
    return r


def config3_check(gold, n_edges, out, gnet, obj, grad):
    """A p=2 batch's results against the stored oracle values: <Z_u Z_v> on 32
    sampled (edge, set) pairs and d<Z_u Z_v>/d(params) on 2 of them; and the
    objective and its gradient against the per-network results they combine
    (obj = |E|/2 - sum Re / 2, grad = -sum grad_net / 2)."""
    o, gn, ob, gr = out.cpu().numpy(), gnet.cpu().numpy(), obj.cpu().numpy(), grad.cpu().numpy()
    err_zz = max(abs(o[i, s, 0] - v) for i, s, v in gold["values"])
    err_g = max(float(np.max(np.abs(gn[i, s] - np.array(g)))) for i, s, g in gold["grads"])
    err_obj = float(np.max(np.abs(ob - (n_edges / 2 - 0.5 * o[:, :, 0].sum(axis=0)))))
    err_gsum = float(np.max(np.abs(gr + 0.5 * gn.sum(axis=0))))
    ok = err_zz <= TOL_ZZ_BF16 and err_g <= TOL_G_BF16 and err_obj <= 1e-9 * n_edges and err_gsum <= 1e-9 * n_edges
    return {"max_abs_zz_vs_oracle": float(err_zz), "max_abs_grad_vs_parameter_shift": err_g,
            "obj_vs_values": err_obj, "grad_vs_grad_net": err_gsum,
            "pairs_checked": len(gold["values"]), "grads_checked": len(gold["grads"]),
            "tolerance": {"zz": TOL_ZZ_BF16, "grad": TOL_G_BF16}, "ok": bool(ok)}


P1_N, P1_D = 100, 3  # the 3-regular n=100 p=1 batch (plain path, batched p=1 row, rows past the hot path)


def next_rows(model, params, edges, st, dev, refs):
    """Rows past the hot path, on the 3-regular n=100 p=1 batch: angle
    optimisation on the adjoint gradient, answer-string estimation, the
    batched pass with noise channels and with diagonal gates."""
    N_VERT, P_LAYERS = P1_N, 1
    import torch
    import workloads
    from paper_1709_03636_amd import answer, noise, optimize, qaoa, qtn
    res = {}
    # angle optimisation: Adam on the batched fwd+grad pass, all 64 starts at once
    steps = 100
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xb, fb, trace = optimize.adam_maximize(lambda x: model.value_and_grad(x), params, steps=steps, lr=0.05)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k = int(fb.argmax())
    best = xb[k].cpu().numpy()
    res["angle_optimisation"] = {
        "workload": f"Adam ascent of <C>, QAOA p=1 on the 3-regular n=100 graph, {params.shape[0]} starts at once",
        "steps": steps, "ms_per_iteration": dt / (steps + 1) * 1e3, "start_best_cost": float(trace[0]),
        "final_best_cost": float(fb[k]), "edges": len(edges), "best_angles": best.tolist()}
    log(f"optimisation: {res['angle_optimisation']}")

    # answer strings: the paper's 30-vertex 3-regular setting (timed) and n=20 graphs against brute force
    def plus(n):
        return np.array([complex(qaoa.PLUS[0], qaoa.PLUS[1]), complex(qaoa.PLUS[2], qaoa.PLUS[3])] * n)

    def opt_angles(n, e):
        m = qaoa.MaxCut(n, e, 1, qtn.TN_C64, order="linegraph", max_sets=16, trials=4)
        x0 = torch.tensor(workloads.qaoa_angles(11, 16, 1), dtype=torch.float64, device=dev)
        xb, fb, _ = optimize.adam_maximize(m.value_and_grad, x0, steps=150, lr=0.05)
        j = int(fb.argmax())
        return xb[j].cpu().numpy(), float(fb[j])

    n30 = 30
    e30 = workloads.random_regular_graph(3, n30, GRAPH_SEED)
    ang30, c30 = opt_angles(n30, e30)
    t0 = time.perf_counter()
    bits, _ = answer.answer_string(n30, qaoa.qaoa_gates(n30, e30, 1), init=plus(n30), n_params=2, params=ang30,
                                   dtype=qtn.TN_C64, tie_tol=1e-4)
    dt30 = time.perf_counter() - t0
    ratios = []
    for seed in range(5):
        e20 = workloads.random_regular_graph(3, 20, seed)
        a20, _ = opt_angles(20, e20)
        b20, _ = answer.answer_string(20, qaoa.qaoa_gates(20, e20, 1), init=plus(20), n_params=2, params=a20,
                                      dtype=qtn.TN_C64, tie_tol=1e-4)
        ratios.append(answer.cut_value(e20, b20) / max_cut_brute_force(20, e20))
    res["answer_string"] = {
        "workload": "qubit-by-qubit projection (one PROBABILITY contraction per qubit, plain path), QAOA p=1 at "
                    "optimised angles, complex64",
        "n30": {"edges": len(e30), "contractions": n30, "seconds": dt30, "cut": answer.cut_value(e30, bits),
                "expected_cut_at_angles": c30},
        "n20_approx_ratio_vs_brute_force": {"graphs": 5, "mean": float(np.mean(ratios)), "min": float(min(ratios))}}
    log(f"answer string: {res['answer_string']}")

    # noise: depolarizing channel after every gate, same batch shape, fwd+grad
    nm = qaoa.MaxCut(N_VERT, edges, P_LAYERS, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=4,
                     noise=noise.depolarizing(0.01))
    nm.batch.autotune(params, reps=10, stream=st)
    for _ in range(5):
        nm.batch.grad(params, stream=st)
    nm.batch.kernel_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    ev0.record(st)
    for _ in range(reps):
        nm.batch.grad(params, stream=st)
    ev1.record(st)
    torch.cuda.synchronize()
    n_t, k_ms = nm.batch.kernel_time(0)
    nm.batch.kernel_timing(False)
    ms = ev0.elapsed_time(ev1) / reps
    ninfo = nm.batch.info()
    res["noise"] = {
        "workload": "the p=1 batch with a depolarizing channel (p = 0.01) after every gate on each of its qubits "
                    "(folded superoperator tensors, light cone kept: trace preserving)",
        "fwd_grad_networks_per_s": len(edges) * N_SETS / (ms * 1e-3), "ms_per_pass": ms,
        "fused_kernel_us": k_ms / max(1, n_t) * 1e3, "n_programs": ninfo["n_programs"]}
    log(f"noise: {res['noise']}")

    # diagonal gates as hyperedge tensors: the p=1 batch, and whole-circuit networks
    dm = qaoa.MaxCut(N_VERT, edges, P_LAYERS, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=4,
                     diagonal=True)
    dm.batch.autotune(params, reps=10, stream=st)
    out = torch.empty((len(edges), N_SETS, 2), dtype=torch.float64, device=dev)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2 * P_LAYERS), dtype=torch.float64, device=dev)
    dm.batch.grad(params, out=out, obj=obj, grad=grad, stream=st)
    st.synchronize()
    ang = params.cpu().numpy()
    err = p1_errors(refs["d3_n100_p1"], out)["max_abs_zz"]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    timed = {}
    for wg in (True, False):
        for _ in range(5):
            dm.batch.run_graph(wg, params, obj=obj, grad=grad if wg else None, stream=st)
        ev0.record(st)
        for _ in range(50):
            dm.batch.run_graph(wg, params, obj=obj, grad=grad if wg else None, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        timed[wg] = ev0.elapsed_time(ev1) / 50
    dm.batch.kernel_timing(True)
    for _ in range(20):
        dm.batch.grad(params, stream=st)
    n_t, k_ms = dm.batch.kernel_time(0)
    dm.batch.kernel_timing(False)
    dinfo = dm.batch.info()
    whole = {}
    for dd, dn in ((6, 20), (6, 30)):
        de = workloads.random_regular_graph(dd, dn, GRAPH_SEED)
        net = qaoa.edge_network(dn, de, 1, de[0], dtype=qtn.TN_C64, lightcone=False, diagonal=True)
        net.set_order(net.order_linegraph(trials=8, seed=0))
        pinfo = net.plan_info()
        a0 = ang[0]
        v = net.contract(a0, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            v = net.contract(a0, stream=st)
        ms = (time.perf_counter() - t0) / 3 * 1e3
        zz_ref = refs["whole_circuit_edge0_set0"][f"d{dd}_n{dn}"]["zz_edge0"]
        whole[f"d{dd}_n{dn}"] = {"peak_bits": pinfo["peak_bits"], "flops": pinfo["flops"], "bytes": pinfo["bytes"],
                                 "ms_per_contraction": ms, "abs_err_zz_vs_closed_form": abs(v.real - zz_ref)}
    res["diagonal"] = {
        "workload": "the p=1 batch with ZZ gates as 16-entry diagonal tensors on hyperedge wires "
                    "(exact; the paper keeps gates dense), complex64",
        "fwd_grad_networks_per_s": len(edges) * N_SETS / (timed[True] * 1e-3), "ms_per_step": timed[True],
        "fwd_networks_per_s": len(edges) * N_SETS / (timed[False] * 1e-3), "ms_per_step_fwd": timed[False],
        "fused_kernel_us": k_ms / max(1, n_t) * 1e3, "max_abs_err_zz": err,
        "flops_fwd_per_set": dinfo["flops_fwd"], "bytes_fwd_per_set": dinfo["bytes_fwd"],
        "whole_circuit_one_edge": whole}
    log(f"diagonal: {res['diagonal']}")
    return res


def batching_grid(st, dev, refs, cases=None):
    """The batching configurations: seeded random 4- and 5-regular graphs with
    n in {50, 70, 100}, p in {1, 2}; all edge light-cone networks x 64 angle
    sets per batch, forward + adjoint gradient from a captured graph, complex64
    with split-BF16 matrix-core products (FP32 accumulation). Also the same
    batches with the diagonal gates on hyperedge wires. Error against the FP64
    oracle (stored values): closed form on every edge of 4 angle sets at p = 1,
    the oracle's light-cone contraction on 64 sampled (edge, set) pairs and the
    parameter-shift gradient on 4 of them at p = 2, checked on the last
    replay."""
    import torch
    import workloads
    from paper_1709_03636_amd import qaoa, qtn
    rows = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p1 = {(b["d"], b["n"]): b for b in refs["grid_p1"]}
    for d in (4, 5):
        for n in (50, 70, 100):
            for p in (1, 2):
                if cases is not None and (d, n, p) not in cases:
                    continue
                e = workloads.random_regular_graph(d, n, GRAPH_SEED)
                ang = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, p))
                prm = torch.tensor(ang, dtype=torch.float64, device=dev)
                row = {"d": d, "n": n, "p": p, "edges": len(e)}
                for mode in ("dense", "diagonal"):
                    m = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=GRID_TRIALS[p],
                                    diagonal=mode == "diagonal")
                    m.batch.set_precision(qtn.TN_MFMA_BF16X3)
                    m.batch.autotune(prm, reps=2, stream=st)
                    out = torch.empty((len(e), N_SETS, 2), dtype=torch.float64, device=dev)
                    gnet = torch.empty((len(e), N_SETS, 2 * p), dtype=torch.float64, device=dev)
                    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
                    grad = torch.empty((N_SETS, 2 * p), dtype=torch.float64, device=dev)
                    t = {}
                    for wg in (False, True):
                        def rep():
                            m.batch.run_graph(wg, prm, out=out, obj=obj, grad=grad if wg else None,
                                              grad_net=gnet if wg else None, stream=st)
                        for _ in range(2):
                            rep()
                        reps = 3
                        ev0.record(st)
                        for _ in range(reps):
                            rep()
                        ev1.record(st)
                        torch.cuda.synchronize()
                        t[wg] = ev0.elapsed_time(ev1) / reps
                    if p == 1:
                        chk = p1_errors(p1[(d, n)], out, gnet)
                    else:
                        chk = config3_check(refs["config3_p2"][(d, n)], len(e), out, gnet, obj, grad)
                    ms = t[True]
                    inf = m.batch.info()
                    row[mode] = {"ms_per_step": ms, "fwd_grad_networks_per_s": len(e) * N_SETS / (ms * 1e-3),
                                 "ms_per_step_fwd": t[False],
                                 "fwd_networks_per_s": len(e) * N_SETS / (t[False] * 1e-3),
                                 "check_vs_oracle": chk,
                                 "executors": {"lds_fused": inf["n_fused"], "global_arena": inf["n_global"],
                                               "level": inf["n_level"], "level_task_groups": inf["n_level_tasked"]},
                                 "flops_per_set": inf["flops_fwd"] + inf["flops_grad"]}
                    del m
                rows.append(row)
                log(f"batching grid: {row}")
    return {"workload": "all edge light-cone networks x 64 angle sets, fwd + adjoint grad, graph replay, complex64 "
                        "with split-BF16 matrix-core products; diagonal: ZZ gates on hyperedge wires",
            "oracle_check": "stored FP64 oracle values: closed form on every edge of 4 angle sets (p=1); light-cone "
                            "contraction on 64 sampled (edge, set) pairs and parameter shift on 4 (p=2); last replay",
            "rows": rows}


def differentiation(st, dev, refs):
    """QAOA p=2 on the seeded 3-regular graph with 60 vertices (90 edge
    networks) x 64 angle sets: forward + adjoint gradient from a captured
    graph, complex64; error of <C> on 4 sets against light-cone state vectors
    and of the gradient on one set against the parameter-shift rule (stored
    oracle values)."""
    import torch
    import workloads
    from paper_1709_03636_amd import qaoa, qtn
    n, p = 60, 2
    e = workloads.random_regular_graph(3, n, GRAPH_SEED)
    ang = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, p))
    prm = torch.tensor(ang, dtype=torch.float64, device=dev)
    m = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=4)
    m.batch.autotune(prm, reps=5, stream=st)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2 * p), dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    timed = {}
    for wg in (True, False):
        for _ in range(5):
            m.batch.run_graph(wg, prm, obj=obj, grad=grad if wg else None, stream=st)
        ev0.record(st)
        for _ in range(20):
            m.batch.run_graph(wg, prm, obj=obj, grad=grad if wg else None, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        timed[wg] = ev0.elapsed_time(ev1) / 20
    m.batch.run_graph(True, prm, obj=obj, grad=grad, stream=st)
    torch.cuda.synchronize()
    ob, gr = obj.cpu().numpy(), grad.cpu().numpy()
    r = refs["d3_n60_p2"]
    err_c = max(abs(ob[s] - c) / c for s, c in zip(r["cost_sets"], r["cost"]))
    ps = np.array(r["grad"])
    err_g = float(np.max(np.abs(gr[r["grad_set"]] - ps)) / max(1.0, np.abs(ps).max()))
    info = m.batch.info()
    res = {"workload": "QAOA p=2 Max-Cut, random 3-regular n=60 (90 edge light-cone networks) x 64 angle sets, "
                       "fwd + adjoint gradient (4 entries), complex64, graph replay",
           "ms_per_step": timed[True], "fwd_grad_networks_per_s": len(e) * N_SETS / (timed[True] * 1e-3),
           "ms_per_step_fwd": timed[False], "fwd_networks_per_s": len(e) * N_SETS / (timed[False] * 1e-3),
           "max_rel_err_cost_vs_statevector": err_c, "rel_err_grad_vs_parameter_shift": err_g,
           "executors": {"lds_fused": info["n_fused"], "global_arena": info["n_global"], "level": info["n_level"]},
           "n_programs": info["n_programs"]}
    log(f"differentiation: {res}")
    return res


def crossover(st, dev, refs):
    """Tensor-network contraction against Hilbert-space simulation, QAOA p=1 on
    seeded random d-regular graphs with 30 vertices, d = 3..7 (the paper's
    crossover in degree): time per <C> (all edges) of the full complex64 state
    vector on this GPU, of the batched light-cone networks (one angle set),
    and of the whole-circuit folded networks (dense and diagonal gates) where
    their largest intermediate stays within 2^30 entries (edge 0 timed, times
    |E|; line-graph orders from 1024 restarts for the dense networks at
    n = 30, 256 otherwise; forward + gradient too at 2^26 entries and up);
    n = 40 for the light-cone networks, where the state vector (8 TiB) does
    not fit, and the order search of the whole-circuit ones. Errors against
    the stored closed-form values."""
    import torch
    import workloads
    from paper_1709_03636_amd import qaoa, qtn
    g0, b0 = 0.4, 0.3
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = None
    rows = []
    for n in (30, 40):
        for d in (3, 4, 5, 6, 7):
            e = workloads.random_regular_graph(d, n, GRAPH_SEED)
            cr = next(r for r in refs["crossover_g0.4_b0.3"] if r["d"] == d and r["n"] == n)
            ref = cr["cost"]
            row = {"d": d, "n": n, "edges": len(e), "cost_closed_form": ref}
            if n <= 30:
                need = qtn.lib().tn_sv_workspace_bytes(n)
                if ws is None or ws.numel() < need:
                    ws = torch.empty(need, dtype=torch.uint8, device=dev)
                v = qtn.sv_maxcut_p1(n, e, g0, b0, workspace=ws, stream=st)
                t0 = time.perf_counter()
                for _ in range(3):
                    v = qtn.sv_maxcut_p1(n, e, g0, b0, workspace=ws, stream=st)
                row["state_vector"] = {"ms_per_cost": (time.perf_counter() - t0) / 3 * 1e3, "abs_err": abs(v - ref),
                                       "bytes": 8 * 2 ** n, "hbm_passes": -(-n // 5)}
            else:
                row["state_vector"] = {"infeasible": f"2^{n} complex64 amplitudes = {8 * 2 ** n / 2 ** 40:.0f} TiB"}
            m = qaoa.MaxCut(n, e, 1, qtn.TN_C64, order="linegraph", max_sets=1, trials=4)
            prm = torch.tensor([[g0, b0]], dtype=torch.float64, device=dev)
            obj = torch.empty(1, dtype=torch.float64, device=dev)
            for _ in range(3):
                m.batch.run_graph(False, prm, obj=obj, stream=st)
            ev0.record(st)
            for _ in range(20):
                m.batch.run_graph(False, prm, obj=obj, stream=st)
            ev1.record(st)
            torch.cuda.synchronize()
            row["tn_lightcone"] = {"ms_per_cost": ev0.elapsed_time(ev1) / 20, "abs_err": abs(obj.item() - ref)}
            # whole-circuit networks (config 5): line-graph order, best of 1024 restarts at n=30 and of 256
            # at n=40 (the order search is anytime; the paper ran QuickBB for 3000 s per circuit)
            for mode in ("dense", "diagonal"):
                trials = 1024 if n <= 30 and mode == "dense" else 256
                net = qaoa.edge_network(n, e, 1, e[0], dtype=qtn.TN_C64, lightcone=False,
                                        diagonal=mode == "diagonal")
                t0 = time.perf_counter()
                pi_order = net.order_linegraph(trials=trials, seed=0)
                search_s = time.perf_counter() - t0
                try:
                    net.set_order(pi_order)
                except qtn.QtnError as ex:  # the order's largest intermediate passes the 2^31-entry cap
                    row[f"tn_whole_circuit_{mode}"] = {"order_restarts": trials, "order_search_s": search_s,
                                                       "infeasible": str(ex)}
                    continue
                pi = net.plan_info()
                r = {"order_restarts": trials, "order_search_s": search_s, "peak_bits": pi["peak_bits"],
                     "flops_per_edge": pi["flops"]}
                if n <= 30 and pi["peak_bits"] <= 30 and pi["flops"] <= 1e14:
                    b = qtn.Batch([net], max_sets=1)
                    prm = torch.tensor([[g0, b0]], dtype=torch.float64, device=dev)
                    out = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
                    b.contract(prm, out=out, stream=st)
                    torch.cuda.synchronize()
                    ev0.record(st)
                    b.contract(prm, out=out, stream=st)
                    ev1.record(st)
                    torch.cuda.synchronize()
                    ms = ev0.elapsed_time(ev1)
                    r.update({"ms_per_edge": ms, "ms_per_cost_estimate": ms * len(e),
                              "tflops": pi["flops"] / (ms * 1e-3) / 1e12,
                              "frac_of_fp32_matrix_peak": pi["flops"] / (ms * 1e-3) / FP32_MFMA_PEAK,
                              "abs_err_zz_edge0": abs(out[0, 0, 0].item() - cr["zz_edge0"])})
                    if pi["peak_bits"] >= 26 and mode == "dense":
                        gn = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
                        ev0.record(st)
                        b.grad(prm, out=out, grad_net=gn, stream=st)
                        ev1.record(st)
                        torch.cuda.synchronize()
                        gms = ev0.elapsed_time(ev1)
                        bi = b.info()
                        r["fwd_grad"] = {"ms_per_edge": gms,
                                         "tflops": (bi["flops_fwd"] + bi["flops_grad"]) / (gms * 1e-3) / 1e12,
                                         "grad": gn[0, 0].cpu().numpy().tolist(),
                                         "abs_err_zz_edge0": abs(out[0, 0, 0].item() - cr["zz_edge0"])}
                    del b
                    torch.cuda.empty_cache()
                elif n > 30:
                    r["not_run"] = "n=40 rows report the order search only"
                else:
                    r["infeasible"] = "largest intermediate beyond 2^30 entries or work beyond 1e14 flops"
                row[f"tn_whole_circuit_{mode}"] = r
                del net
            rows.append(row)
            log(f"crossover: {row}")
    return {"workload": "QAOA p=1 Max-Cut <C>, random d-regular graphs, gamma=0.4, beta=0.3; time per <C> over all "
                        "edges; state vector: full 2^n complex64 on this GPU",
            "rows": rows}


def executor_rooflines(model, params, st, steps, n_sets, prec_name):
    """Each executor's kernel on eager passes (HIP events around each launch,
    on its stream): average duration, algorithmic rates and roofline figures.
    Level (task executor): bound by the matrix cores, priced at the executed
    precision (split-BF16: three bf16 products per real product), with the
    FP32-equivalent rate beside it. Fused executors (thin contractions on the
    vector units, operands in LDS or L2): bound by vector instruction issue,
    priced against the FP32 vector peak."""
    import torch
    from paper_1709_03636_amd import qtn
    info = model.batch.info()
    for _ in range(2):
        model.batch.grad(params, stream=st)
    torch.cuda.synchronize()
    model.batch.kernel_timing(True)
    for _ in range(steps):
        model.batch.grad(params, stream=st)
    torch.cuda.synchronize()
    res = {}
    names = {qtn.TN_EXEC_FUSED: "lds_fused", qtn.TN_EXEC_LEVEL: "level", qtn.TN_EXEC_GLOBAL: "global_arena"}
    for ex, name in names.items():
        n_t, total = model.batch.kernel_time(ex)
        if n_t == 0:
            continue
        ms = total / n_t
        flops = info["exec_flops"][ex] * n_sets
        byts = info["exec_bytes"][ex] * n_sets
        r = {"launches_timed": n_t, "kernel_ms": ms, "algorithmic_flops_per_launch": flops,
             "algorithmic_bytes_per_launch": byts, "fp32_equiv_tflops": flops / (ms * 1e-3) / 1e12}
        if ex == qtn.TN_EXEC_LEVEL:
            # the binding roofline: the larger of the HBM time of the algorithmic bytes and the
            # matrix-core time of the executed products (split-BF16: three per real product)
            mf = info["level_mfma_flops"] * n_sets
            mult, peak = (3.0, BF16_MFMA_PEAK) if prec_name == "bf16x3" else (1.0, FP32_MFMA_PEAK)
            if prec_name == "fp64":
                peak = FP64_MFMA_PEAK
            t_hbm, t_mfma = byts / HBM_PEAK, mult * mf / peak
            ach_m = mult * mf / (ms * 1e-3)
            r.update({"matrix_core_share_of_flops": mf / max(flops, 1.0), "executed_precision": prec_name,
                      "ideal_ms_hbm": t_hbm * 1e3, "ideal_ms_mfma": t_mfma * 1e3,
                      "mfma_executed_tflops": ach_m / 1e12, "mfma_frac": ach_m / peak,
                      "hbm_frac": byts / (ms * 1e-3) / HBM_PEAK,
                      "fp32_equiv_frac_of_fp32_matrix_peak": flops / (ms * 1e-3) / FP32_MFMA_PEAK})
            if t_hbm >= t_mfma:
                r.update({"bound": "hbm", "achieved": byts / (ms * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                          "unit": "GB/s", "frac": byts / (ms * 1e-3) / HBM_PEAK})
            else:
                r.update({"bound": "mfma", "achieved": ach_m / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                          "frac": ach_m / peak})
        else:
            ach = flops / (ms * 1e-3)
            r.update({"bound": "alu", "achieved": ach / 1e12, "peak": FP32_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                      "frac": ach / FP32_VALU_PEAK, "algorithmic_gbps": byts / (ms * 1e-3) / 1e9})
        res[name] = r
    model.batch.kernel_timing(False)
    return res


def headline(args, st, dev, refs):
    """The timed step on the headline workload, its post-timing oracle check,
    and the executors' kernel figures."""
    import torch
    import workloads
    from paper_1709_03636_amd import qtn, qaoa
    d, n, p = HEAD_D, HEAD_N, HEAD_P
    edges = workloads.random_regular_graph(d, n, GRAPH_SEED)
    angles = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, p))
    n_nets = len(edges)
    log(f"headline: d={d} n={n} p={p} edges={n_nets} sets={N_SETS}")
    t0 = time.perf_counter()
    model = qaoa.MaxCut(n, edges, p, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=GRID_TRIALS[p])
    plan_s = time.perf_counter() - t0
    model.batch.set_precision(qtn.TN_MFMA_BF16X3)
    params = torch.tensor(angles, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    model.batch.autotune(params, reps=2, stream=st)
    st.synchronize()
    tune_s = time.perf_counter() - t0
    info = model.batch.info()
    log(f"planned in {plan_s:.1f}s, autotuned in {tune_s:.1f}s: {info}")
    out = torch.empty((n_nets, N_SETS, 2), dtype=torch.float64, device=dev)
    gnet = torch.empty((n_nets, N_SETS, 2 * p), dtype=torch.float64, device=dev)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2 * p), dtype=torch.float64, device=dev)

    def replay(with_grad):
        model.batch.run_graph(with_grad, params, out=out, obj=obj, grad=grad if with_grad else None,
                              grad_net=gnet if with_grad else None, stream=st)

    for _ in range(args.warmup):
        replay(True)
    torch.cuda.synchronize()
    out.fill_(float("nan"))
    gnet.fill_(float("nan"))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(st)
    for _ in range(args.steps):
        replay(True)
    ev1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n_nets * N_SETS / (ms_step * 1e-3)
    log(f"fwd+grad: {ms_step:.3f} ms/step, {value:.4e} networks/s (wall {wall:.3f}s for {args.steps} steps)")
    # the last timed replay's results against the oracle
    check = config3_check(refs["config3_p2"][(d, n)], n_nets, out, gnet, obj, grad)
    log(f"post-timing check: {check}")
    # forward only
    for _ in range(args.warmup):
        replay(False)
    ev0.record(st)
    for _ in range(args.steps):
        replay(False)
    ev1.record(st)
    torch.cuda.synchronize()
    ms_fwd = ev0.elapsed_time(ev1) / args.steps
    log(f"fwd: {ms_fwd:.3f} ms/step")
    kern = executor_rooflines(model, params, st, max(3, min(args.steps, 10)), N_SETS, "bf16x3")
    log(f"executor kernels: {kern}")
    return {"value": value, "ms_per_step": ms_step, "wall_s": wall, "ms_per_step_fwd": ms_fwd,
            "fwd_networks_per_s": n_nets * N_SETS / (ms_fwd * 1e-3), "n_nets": n_nets, "check": check,
            "kernels": kern, "info": info, "plan_s": plan_s, "autotune_s": tune_s, "edges": edges,
            "angles": angles}


def p1_rows(args, st, dev, refs):
    """The 3-regular n=100 p=1 batch x 64 angle sets: batched fwd+grad (graph
    replay, FP32 products), its fused kernel's figures, and the plain path
    (one network per launch) in complex64 and complex128."""
    import torch
    import workloads
    from paper_1709_03636_amd import qtn, qaoa
    n, p = P1_N, 1
    edges = workloads.random_regular_graph(P1_D, n, GRAPH_SEED)
    angles = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, p))
    model = qaoa.MaxCut(n, edges, p, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=GRID_TRIALS[p])
    params = torch.tensor(angles, dtype=torch.float64, device=dev)
    model.batch.autotune(params, reps=10, stream=st)
    info = model.batch.info()
    out = torch.empty((len(edges), N_SETS, 2), dtype=torch.float64, device=dev)
    gnet = torch.empty((len(edges), N_SETS, 2), dtype=torch.float64, device=dev)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2), dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    timed = {}
    for wg in (True, False):
        def rep():
            model.batch.run_graph(wg, params, out=out, obj=obj, grad=grad if wg else None,
                                  grad_net=gnet if wg else None, stream=st)
        for _ in range(5):
            rep()
        ev0.record(st)
        for _ in range(args.steps):
            rep()
        ev1.record(st)
        torch.cuda.synchronize()
        timed[wg] = ev0.elapsed_time(ev1) / args.steps
        if wg:
            chk = p1_errors(refs["d3_n100_p1"], out, gnet, obj, grad)
    kern = executor_rooflines(model, params, st, args.steps, N_SETS, "fp32")
    if info["sets_per_wave_grad"] > 1:
        kname = f"fused_sets_kernel<float, true, {6 - info['sets_per_wave_grad'] // 2}>"
    else:
        kname = (f"fused_exec_kernel<float, {info['fused_block']}, true, "
                 f"{'true' if info['rec_only'] & 2 else 'false'}, false>")
    if "lds_fused" in kern:
        kern["lds_fused"]["kernel"] = kname
        kern["lds_fused"]["bound_note"] = ("operands stay in LDS (HBM traffic is a small fraction of the "
                                           "algorithmic bytes); the limiter is vector instruction issue")
        kern["lds_fused"]["traffic"] = traffic_from_profile("fused_exec_grad.qaoa_d3_n100_p1_s64", kname)
    batched = {"workload": f"QAOA p=1 Max-Cut, random 3-regular graph n={n} ({len(edges)} edge light-cone networks) "
                           f"x {N_SETS} angle sets, fwd + adjoint grad, complex64 (FP32), graph replay",
               "ms_per_step": timed[True], "fwd_grad_networks_per_s": len(edges) * N_SETS / (timed[True] * 1e-3),
               "ms_per_step_fwd": timed[False], "fwd_networks_per_s": len(edges) * N_SETS / (timed[False] * 1e-3),
               "check_vs_closed_form": chk, "kernels": kern}
    log(f"p=1 batch: {batched}")
    # plain path: one network per launch, complex64 and complex128 (host sync per network)
    plain = {}
    blk = refs["d3_n100_p1"]
    for name, dt in (("c64", qtn.TN_C64), ("c128", qtn.TN_C128)):
        nets = qaoa.edge_networks(n, edges, p, dt, order="linegraph", trials=4)
        a0 = angles[0]
        for net in nets:  # plan-time device set-up of every network, outside the timed loops
            net.contract(a0, stream=st)
            net.grad(a0, stream=st)
        t0 = time.perf_counter()
        vals = [net.contract(a0, stream=st) for net in nets]
        dtp = time.perf_counter() - t0
        t0 = time.perf_counter()
        grads = [net.grad(a0, stream=st) for net in nets]
        dtg = time.perf_counter() - t0
        zz = np.array(blk["zz"][blk["sets"].index(0)])
        dzz = np.array(blk["dzz"][blk["sets"].index(0)])
        gerr = max(float(np.max(np.abs(g - dzz[i]))) for i, (_, g) in enumerate(grads))
        plain[name] = {"networks_per_s": len(nets) / dtp,
                       "max_abs_err_zz": float(np.max(np.abs(np.array(vals).real - zz))),
                       "fwd_grad_networks_per_s": len(nets) / dtg, "max_abs_err_grad": gerr}
        log(f"plain {name}: {plain[name]}")
    return model, params, edges, angles, batched, plain


def dense_row(st, dev, refs, angles):
    """The dense regime on the matrix cores: the whole-circuit network of one
    edge, 6-regular n=20, p=1 (no light cone), FP32 4M, split-BF16 and FP64
    products."""
    import torch
    import workloads
    from paper_1709_03636_amd import qtn, qaoa
    dd, dn = 6, 20
    ref = refs["whole_circuit_edge0_set0"][f"d{dd}_n{dn}"]
    de = workloads.random_regular_graph(dd, dn, GRAPH_SEED)
    a0 = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, 1))[0]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ev0.record(st)
        for _ in range(reps):
            fn()
        ev1.record(st)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    dnet = qaoa.edge_network(dn, de, 1, de[0], dtype=qtn.TN_C64, lightcone=False)
    dnet.set_order(dnet.order_linegraph(trials=8, seed=0))
    dinfo = dnet.plan_info()
    dbatch = qtn.Batch([dnet], max_sets=1)
    dpar = torch.tensor([a0], dtype=torch.float64, device=dev)
    dbatch.autotune(dpar, reps=2, stream=st)
    dout = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
    d_ms = timed(lambda: dbatch.contract(dpar, out=dout, stream=st))
    v32 = dout[0, 0, 0].item()
    dgn = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
    doutg = torch.empty_like(dout)
    g_ms = timed(lambda: dbatch.grad(dpar, out=doutg, grad_net=dgn, stream=st))
    dbi = dbatch.info()
    g_flops = dbi["flops_fwd"] + dbi["flops_grad"]
    g_err = float(np.max(np.abs(dgn[0, 0].cpu().numpy() - np.array(ref["dzz_edge0"]))))
    dbatch.set_precision(qtn.TN_MFMA_BF16X3)
    dbatch.autotune(dpar, reps=2, stream=st)
    dout2 = torch.empty_like(dout)
    b_ms = timed(lambda: dbatch.contract(dpar, out=dout2, stream=st))
    dnet128 = qaoa.edge_network(dn, de, 1, de[0], dtype=qtn.TN_C128, lightcone=False)
    dnet128.set_order(dnet128.order_linegraph(trials=8, seed=0))
    dbatch128 = qtn.Batch([dnet128], max_sets=1)
    dbatch128.autotune(dpar, reps=2, stream=st)
    dout3 = torch.empty_like(dout)
    f_ms = timed(lambda: dbatch128.contract(dpar, out=dout3, stream=st))
    zz_ref = ref["zz_edge0"]
    mfma = {"workload": f"whole-circuit folded network of one edge, QAOA p=1, {dd}-regular n={dn} "
                        f"(no light cone), line-graph order, complex64, 4M FP32 matrix-core products",
            "peak_bits": dinfo["peak_bits"], "flops_per_pass": dinfo["flops"], "pass_ms": d_ms,
            "tflops": dinfo["flops"] / (d_ms * 1e-3) / 1e12,
            "frac_of_fp32_matrix_peak": dinfo["flops"] / (d_ms * 1e-3) / FP32_MFMA_PEAK,
            "abs_err_zz_vs_closed_form": abs(v32 - zz_ref),
            "fwd_grad": {"pass_ms": g_ms, "flops_per_pass": g_flops, "tflops": g_flops / (g_ms * 1e-3) / 1e12,
                         "frac_of_fp32_matrix_peak": g_flops / (g_ms * 1e-3) / FP32_MFMA_PEAK,
                         "abs_err_grad_vs_closed_form": g_err},
            "split_bf16": {"pass_ms": b_ms, "tflops_fp32_equivalent": dinfo["flops"] / (b_ms * 1e-3) / 1e12,
                           "executed_bf16_frac_of_bf16_peak": 3 * dinfo["flops"] / (b_ms * 1e-3) / BF16_MFMA_PEAK,
                           "abs_err_zz_vs_closed_form": abs(dout2[0, 0, 0].item() - zz_ref)},
            "complex128_fp64": {"pass_ms": f_ms, "tflops": dinfo["flops"] / (f_ms * 1e-3) / 1e12,
                                "frac_of_fp64_matrix_peak": dinfo["flops"] / (f_ms * 1e-3) / FP64_MFMA_PEAK,
                                "abs_err_zz_vs_closed_form": abs(dout3[0, 0, 0].item() - zz_ref)}}
    log(f"dense/MFMA: {mfma}")
    return mfma


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-next", action="store_true", help="skip the optimisation / answer-string / noise lines")
    ap.add_argument("--no-grid", action="store_true", help="skip the batching grid, differentiation and crossover")
    ap.add_argument("--headline-only", action="store_true", help="only the headline measurement (for profiling)")
    ap.add_argument("--extras", action="store_true",
                    help="only the batching grid, differentiation and crossover rows, as one JSON line")
    ap.add_argument("--grid-case", action="append", default=None,
                    help="only this batching-grid row d,n,p (e.g. 5,50,2; repeatable); prints the rows as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note "
                                   "(independent networks, one FP64 all-reduce), not implemented"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.steps)
        return

    import torch

    dev = torch.device("cuda:0")
    refs = load_refs()
    if args.grid_case:
        cases = {tuple(int(x) for x in c.split(",")) for c in args.grid_case}
        print(json.dumps(batching_grid(torch.cuda.Stream(), dev, refs, cases=cases)), flush=True)
        return
    if args.extras:
        st = torch.cuda.Stream()
        print(json.dumps({"batching_grid": batching_grid(st, dev, refs),
                          "differentiation_p2_n60": differentiation(st, dev, refs),
                          "crossover_in_degree": crossover(st, dev, refs)}), flush=True)
        return
    st = torch.cuda.Stream()
    h = headline(args, st, dev, refs)
    lvl = h["kernels"].get("level")
    dom_name = max(h["kernels"], key=lambda k: h["kernels"][k]["kernel_ms"])
    dom = h["kernels"][dom_name]
    roofline = {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roofline.update({"kernel": {"level": "task_kernel<2> (task executor, split-BF16)",
                                "global_arena": "fused_exec_kernel<float, 256, true, false, true>",
                                "lds_fused": "fused executor"}[dom_name],
                     "executor": dom_name, "kernel_ms": dom["kernel_ms"], "launches_timed": dom["launches_timed"],
                     "algorithmic_flops_per_launch": dom["algorithmic_flops_per_launch"],
                     "algorithmic_bytes_per_launch": dom["algorithmic_bytes_per_launch"],
                     "traffic": traffic_from_profile(f"{dom_name}.qaoa_d5_n100_p2_s64",
                                                     roofline_kernel_symbol(dom_name))})
    extra = {k: v for k, v in dom.items() if k not in roofline}
    roofline.update({"detail": extra, "all_executors": h["kernels"]})
    if not args.headline_only:
        p1_model, p1_params, p1_edges, p1_angles, batched, plain = p1_rows(args, st, dev, refs)
        mfma = None if args.no_dense else dense_row(st, dev, refs, p1_angles)
        nxt = None if args.no_next else next_rows(p1_model, p1_params, p1_edges, st, dev, refs)
    else:
        p1_edges = p1_angles = batched = plain = mfma = nxt = None
    grid = diff = cross = None
    if not args.no_grid and not args.headline_only:
        # the other configurations run in a child process (its own GPU context): a failure there is
        # recorded in their entries and does not take the headline measurement with it
        import subprocess
        status = None
        try:
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--extras"], stdout=subprocess.PIPE,
                               text=True, timeout=1200)
            status = r.returncode
            ex = json.loads(r.stdout.strip().splitlines()[-1])
            grid, diff, cross = ex["batching_grid"], ex["differentiation_p2_n60"], ex["crossover_in_degree"]
        except subprocess.TimeoutExpired:
            grid = diff = cross = {"error": "child process killed after 1200 s"}
            log("extras failed: time limit")
        except (ValueError, IndexError, KeyError):
            grid = diff = cross = {"error": f"child process exited with status {status}"}
            log(f"extras failed: exit status {status}")

    cpu = cpu_p1 = None
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        cpu = cpu_baseline(HEAD_N, h["edges"], HEAD_P, h["angles"], 20.0,
                           f"the headline batch (5-regular n={HEAD_N}, p={HEAD_P}, 64 angle sets)")
        cpu["gpu_over_cpu"] = h["value"] / cpu["value"]
        log(f"cpu baseline: {cpu}")
        if p1_edges is not None:
            cpu_p1 = cpu_baseline(P1_N, p1_edges, 1, p1_angles, 6.0,
                                  f"the 3-regular n={P1_N} p=1 batch (64 angle sets)")
            log(f"cpu baseline p=1: {cpu_p1}")

    check = h["check"]
    rec = {
        "metric": "QAOA <ZZ> networks contracted/s (fwd, fwd+grad), FP32 vs FP64 oracle err",
        "value": h["value"],
        "unit": "networks/s (fwd+grad)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (FP32 complex; split-BF16 matrix-core products, FP32 accumulation), FP64 final scalars and "
                 "gradient sums",
        "data": "synthetic (seeded random regular graphs and angle sets)",
        "config": {"workload": f"QAOA Max-Cut p={HEAD_P}, random {HEAD_D}-regular graph n={HEAD_N} "
                               f"({h['n_nets']} edge light-cone networks) x {N_SETS} angle sets, fwd + adjoint grad, "
                               "line-graph order (best of 128 restarts), split-BF16 matrix-core products, "
                               "one hipGraph replay per step",
                   "networks_per_step": h["n_nets"] * N_SETS, "parallelism": "single GPU"},
        "fwd_networks_per_s": h["fwd_networks_per_s"],
        "ms_per_step_fwd": h["ms_per_step_fwd"],
        "error_vs_fp64_oracle": check,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "executors": {"lds_fused": h["info"]["n_fused"], "global_arena": h["info"]["n_global"],
                      "level": h["info"]["n_level"], "level_task_groups": h["info"]["n_level_tasked"]},
        "plan_s": h["plan_s"], "autotune_s": h["autotune_s"],
        "p1_batch_3regular_n100": batched,
        "plain_one_network_per_launch_3regular_n100_p1": plain,
        "cpu_baseline_p1_batch": cpu_p1,
        "mfma_path": mfma,
        "next_rows": nxt,
        "batching_grid": grid,
        "differentiation_p2_n60": diff,
        "crossover_in_degree": cross,
    }
    print(json.dumps(rec), flush=True)
    if not check["ok"]:
        log("headline results outside the oracle tolerance")
        sys.exit(1)


def roofline_kernel_symbol(executor):
    return {"level": "task_kernel<2>", "global_arena": "fused_exec_kernel<float, 256, true, false, true>",
            "lds_fused": "fused_exec_kernel"}[executor]


if __name__ == "__main__":
    main()
