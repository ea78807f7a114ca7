"""Benchmark: batched QAOA <Z_u Z_v> network contraction, forward + adjoint gradient.

Workload: QAOA p=1 Max-Cut on a seeded random 3-regular graph with 100
vertices (150 edges), one folded light-cone network per edge, line-graph
(min-fill) contraction order, complex64 contraction with FP64 final scalars
and gradient sums, 64 angle sets (gamma, beta) uniform in [0, pi) from seed 0.
One step = one pass of the whole path over the batch: angle binding, every
pairwise contraction, the final FP64 scalars, the adjoint sweep and the FP64
objective/gradient combine, replayed from a captured HIP graph.

Prints one JSON line (rank 0). Also measured: forward-only throughput, the
plain one-network-per-launch path in complex64 and complex128, the error
against the closed-form p=1 oracle, the dominant kernel's roofline figures
and the FP64 CPU oracle timed on a bounded sample.
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

D, N_VERT, P_LAYERS, N_SETS, GRAPH_SEED, ANGLE_SEED = 3, 100, 1, 64, 0, 0
# restarts of the line-graph order search per network in the batching grid: at p = 2 on 5-regular
# graphs the best of 128 has 2-4x fewer flops than the best of 4 (plan time, on host threads)
GRID_TRIALS = {1: 4, 2: 128}
HBM_PEAK = 8.0e12
FP32_MFMA_PEAK = 157.3e12
FP64_MFMA_PEAK = 78.6e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_worker(args):
    n, edges, p, edge, params = args
    from oracle import tensornet, gates
    import numpy as np
    # forward plus central finite differences in every parameter (2p)
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


def cpu_baseline(edges, angles, budget_s=12.0):
    """The FP64 oracle (plain tensordot contraction) on a bounded sample."""
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    tasks = []
    for s in range(angles.shape[0]):
        for e in edges:
            tasks.append((N_VERT, edges, P_LAYERS, e, np.array(angles[s])))
    # size the sample from a single-network probe
    t0 = time.perf_counter()
    _oracle_worker(tasks[0])
    one = time.perf_counter() - t0
    n_sample = int(min(len(tasks), max(workers, budget_s * workers / max(one, 1e-4))))
    sample = tasks[:n_sample]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_worker, sample, chunksize=max(1, n_sample // (4 * workers)))
        dt = time.perf_counter() - t0
    # one core: a short sample in this process
    n1 = int(max(4, min(len(tasks), 2.0 / max(one, 1e-4))))
    t0 = time.perf_counter()
    for t in tasks[:n1]:
        _oracle_worker(t)
    dt1 = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "networks/s (fwd+grad)", "cores": workers, "kind": "oracle",
            "value_1core": n1 / dt1,
            "sample": f"{n_sample} (edge, angle-set) networks of the same workload, forward plus central "
                      f"finite-difference gradient (5 FP64 contractions each), {workers} processes; "
                      f"1-core figure from {n1} networks in one process"}


def traffic_from_profile(kernel):
    """HBM bytes per launch of the fused adjoint kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the summary covers
    another kernel instance or the kernel source changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.fused_exec_grad.json")
    src = os.path.join(ROOT, "paper_1709_03636_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_prefix") != sha or rec.get("kernel") != kernel:
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


def next_rows(model, params, edges, st, dev):
    """Rows past the hot path: angle optimisation on the adjoint gradient,
    answer-string estimation, and the batched pass with noise channels."""
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
        "workload": f"Adam ascent of <C>, QAOA p={P_LAYERS} on the headline graph, {params.shape[0]} starts at once",
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
    n_t, k_ms = nm.batch.kernel_time()
    nm.batch.kernel_timing(False)
    ms = ev0.elapsed_time(ev1) / reps
    ninfo = nm.batch.info()
    res["noise"] = {
        "workload": "headline batch with a depolarizing channel (p = 0.01) after every gate on each of its qubits "
                    "(folded superoperator tensors, light cone kept: trace preserving)",
        "fwd_grad_networks_per_s": len(edges) * N_SETS / (ms * 1e-3), "ms_per_pass": ms,
        "fused_kernel_us": k_ms / max(1, n_t) * 1e3, "n_programs": ninfo["n_programs"]}
    log(f"noise: {res['noise']}")

    # diagonal gates as hyperedge tensors: the headline batch, and whole-circuit networks
    from oracle import closed_form
    dm = qaoa.MaxCut(N_VERT, edges, P_LAYERS, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=4,
                     diagonal=True)
    dm.batch.autotune(params, reps=10, stream=st)
    out = torch.empty((len(edges), N_SETS, 2), dtype=torch.float64, device=dev)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2 * P_LAYERS), dtype=torch.float64, device=dev)
    dm.batch.grad(params, out=out, obj=obj, grad=grad, stream=st)
    st.synchronize()
    ang = params.cpu().numpy()
    err = max(float(np.max(np.abs(out[:, s, 0].cpu().numpy() - closed_form.zz_p1(N_VERT, edges, *ang[s]))))
              for s in range(N_SETS))
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
    n_t, k_ms = dm.batch.kernel_time()
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
        whole[f"d{dd}_n{dn}"] = {"peak_bits": pinfo["peak_bits"], "flops": pinfo["flops"], "bytes": pinfo["bytes"],
                                 "ms_per_contraction": ms,
                                 "abs_err_zz_vs_closed_form": abs(v.real - closed_form.zz_p1(dn, de, *a0)[0])}
    res["diagonal"] = {
        "workload": "the headline batch with ZZ gates as 16-entry diagonal tensors on hyperedge wires "
                    "(exact; the paper keeps gates dense), complex64",
        "fwd_grad_networks_per_s": len(edges) * N_SETS / (timed[True] * 1e-3), "ms_per_step": timed[True],
        "fwd_networks_per_s": len(edges) * N_SETS / (timed[False] * 1e-3), "ms_per_step_fwd": timed[False],
        "fused_kernel_us": k_ms / max(1, n_t) * 1e3, "max_abs_err_zz": err,
        "flops_fwd_per_set": dinfo["flops_fwd"], "bytes_fwd_per_set": dinfo["bytes_fwd"],
        "whole_circuit_one_edge": whole}
    log(f"diagonal: {res['diagonal']}")
    return res


def batching_grid(st, dev, cases=None):
    """The batching configurations: seeded random 4- and 5-regular graphs with
    n in {50, 70, 100}, p in {1, 2}; all edge light-cone networks x 64 angle
    sets per batch, forward + adjoint gradient from a captured graph, complex64
    with split-BF16 matrix-core products (FP32 accumulation). Also the same
    batches with the diagonal gates on hyperedge wires. Error against the FP64
    oracle: closed form for every edge and set at p = 1, the oracle's
    light-cone contraction on 4 sampled (edge, set) pairs at p = 2."""
    import torch
    import workloads
    from oracle import closed_form, gates, tensornet
    from paper_1709_03636_amd import qaoa, qtn
    rows = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for d in (4, 5):
        for n in (50, 70, 100):
            for p in (1, 2):
                if cases is not None and (d, n, p) not in cases:
                    continue
                e = workloads.random_regular_graph(d, n, GRAPH_SEED)
                ang = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, p))
                prm = torch.tensor(ang, dtype=torch.float64, device=dev)
                if p == 1:
                    ref = {(i, s): v for s in range(N_SETS)
                           for i, v in enumerate(closed_form.zz_p1(n, e, ang[s, 0], ang[s, 1]))}
                else:
                    rng = workloads.SplitMix64(d * 1000 + n)
                    ref = {}
                    for _ in range(4):
                        i, s = rng.below(len(e)), rng.below(N_SETS)
                        gl = gates.qaoa_gate_list(n, e, ang[s, :p], ang[s, p:])[n:]
                        pauli = [0] * n
                        pauli[e[i][0]] = pauli[e[i][1]] = 3
                        ref[(i, s)] = tensornet.expectation(n, gl, pauli, init=[np.array([1.0, 1.0]) / math.sqrt(2)] * n,
                                                            lightcone=True).real
                row = {"d": d, "n": n, "p": p, "edges": len(e)}
                for mode in ("dense", "diagonal"):
                    m = qaoa.MaxCut(n, e, p, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=GRID_TRIALS[p],
                                    diagonal=mode == "diagonal")
                    m.batch.set_precision(qtn.TN_MFMA_BF16X3)
                    m.batch.autotune(prm, reps=2, stream=st)
                    out = torch.empty((len(e), N_SETS, 2), dtype=torch.float64, device=dev)
                    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
                    grad = torch.empty((N_SETS, 2 * p), dtype=torch.float64, device=dev)
                    m.batch.grad(prm, out=out, obj=obj, grad=grad, stream=st)
                    st.synchronize()
                    o = out.cpu().numpy()
                    err = max(abs(o[i, s, 0] - v) for (i, s), v in ref.items())
                    t = {}
                    for wg in (True, False):
                        for _ in range(2):
                            m.batch.run_graph(wg, prm, obj=obj, grad=grad if wg else None, stream=st)
                        reps = 3
                        ev0.record(st)
                        for _ in range(reps):
                            m.batch.run_graph(wg, prm, obj=obj, grad=grad if wg else None, stream=st)
                        ev1.record(st)
                        torch.cuda.synchronize()
                        t[wg] = ev0.elapsed_time(ev1) / reps
                    ms = t[True]
                    inf = m.batch.info()
                    row[mode] = {"ms_per_step": ms, "fwd_grad_networks_per_s": len(e) * N_SETS / (ms * 1e-3),
                                 "ms_per_step_fwd": t[False],
                                 "fwd_networks_per_s": len(e) * N_SETS / (t[False] * 1e-3),
                                 "max_abs_err_zz": float(err),
                                 "executors": {"lds_fused": inf["n_fused"], "global_arena": inf["n_global"],
                                               "level": inf["n_level"]},
                                 "flops_per_set": inf["flops_fwd"] + inf["flops_grad"]}
                    del m
                rows.append(row)
                log(f"batching grid: {row}")
    return {"workload": "all edge light-cone networks x 64 angle sets, fwd + adjoint grad, graph replay, complex64 "
                        "with split-BF16 matrix-core products; diagonal: ZZ gates on hyperedge wires",
            "oracle_check": "closed form, all edges and sets (p=1); FP64 light-cone contraction, 4 sampled (edge, "
                            "set) pairs (p=2)",
            "rows": rows}


def differentiation(st, dev):
    """QAOA p=2 on the seeded 3-regular graph with 60 vertices (90 edge
    networks) x 64 angle sets: forward + adjoint gradient from a captured
    graph, complex64; error of <C> on every set against light-cone state
    vectors, of the gradient on one set against the parameter-shift rule."""
    import torch
    import workloads
    from oracle import gradients, statevector
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
    err_c = 0.0
    for s in range(0, N_SETS, 16):
        zz = np.array([statevector.qaoa_zz_edge(n, e, ang[s, :p], ang[s, p:], ed) for ed in e])
        c_ref = float(np.sum((1 - zz) / 2))
        err_c = max(err_c, abs(ob[s] - c_ref) / c_ref)
    s = 1
    ps = sum(-0.5 * gradients.parameter_shift_edge(n, e, ang[s], ed) for ed in e)
    err_g = float(np.max(np.abs(gr[s] - ps)) / max(1.0, np.abs(ps).max()))
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


def crossover(st, dev):
    """Tensor-network contraction against Hilbert-space simulation, QAOA p=1 on
    seeded random d-regular graphs with 30 vertices, d = 3..7 (the paper's
    crossover in degree): time per <C> (all edges) of the full complex64 state
    vector on this GPU, of the batched light-cone networks (one angle set),
    and of the whole-circuit folded networks (dense and diagonal gates) where
    their largest intermediate fits (edge 0 timed, times |E|); n = 40 for the
    light-cone networks, where the state vector (8 TiB) does not fit."""
    import torch
    import workloads
    from oracle import closed_form
    from paper_1709_03636_amd import qaoa, qtn
    g0, b0 = 0.4, 0.3
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = None
    rows = []
    for n in (30, 40):
        for d in (3, 4, 5, 6, 7):
            e = workloads.random_regular_graph(d, n, GRAPH_SEED)
            ref = closed_form.cost_p1(n, e, g0, b0)
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
            if n <= 30:
                for mode in ("dense", "diagonal"):
                    net = qaoa.edge_network(n, e, 1, e[0], dtype=qtn.TN_C64, lightcone=False,
                                            diagonal=mode == "diagonal")
                    try:
                        net.set_order(net.order_linegraph(trials=4, seed=0))
                    except qtn.QtnError as ex:  # the order's largest intermediate passes the memory limit
                        row[f"tn_whole_circuit_{mode}"] = {"infeasible": str(ex)}
                        continue
                    pi = net.plan_info()
                    r = {"peak_bits": pi["peak_bits"], "flops_per_edge": pi["flops"]}
                    if pi["peak_bits"] <= 28 and pi["flops"] <= 2e13:
                        net.contract([g0, b0], stream=st)
                        t0 = time.perf_counter()
                        z = net.contract([g0, b0], stream=st)
                        r["ms_per_edge"] = (time.perf_counter() - t0) * 1e3
                        r["ms_per_cost_estimate"] = r["ms_per_edge"] * len(e)
                        r["abs_err_zz_edge0"] = abs(z.real - closed_form.zz_p1(n, e, g0, b0)[0])
                    else:
                        r["infeasible"] = "largest intermediate beyond 2^28 entries or work beyond 2e13 flops"
                    row[f"tn_whole_circuit_{mode}"] = r
                    del net
            rows.append(row)
            log(f"crossover: {row}")
    return {"workload": "QAOA p=1 Max-Cut <C>, random d-regular graphs, gamma=0.4, beta=0.3; time per <C> over all "
                        "edges; state vector: full 2^n complex64 on this GPU",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-next", action="store_true", help="skip the optimisation / answer-string / noise lines")
    ap.add_argument("--no-grid", action="store_true", help="skip the 4-/5-regular batching grid")
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
    import workloads
    from paper_1709_03636_amd import qtn, qaoa

    dev = torch.device("cuda:0")
    if args.grid_case:
        cases = {tuple(int(x) for x in c.split(",")) for c in args.grid_case}
        print(json.dumps(batching_grid(torch.cuda.Stream(), dev, cases=cases)), flush=True)
        return
    if args.extras:
        st = torch.cuda.Stream()
        print(json.dumps({"batching_grid": batching_grid(st, dev), "differentiation_p2_n60": differentiation(st, dev),
                          "crossover_in_degree": crossover(st, dev)}), flush=True)
        return
    edges = workloads.random_regular_graph(D, N_VERT, GRAPH_SEED)
    angles = np.array(workloads.qaoa_angles(ANGLE_SEED, N_SETS, P_LAYERS))
    n_nets = len(edges)
    log(f"workload d={D} n={N_VERT} p={P_LAYERS} edges={n_nets} sets={N_SETS}")

    t0 = time.perf_counter()
    model = qaoa.MaxCut(N_VERT, edges, P_LAYERS, qtn.TN_C64, order="linegraph", max_sets=N_SETS, trials=4)
    info = model.batch.info()
    log(f"plans compiled in {time.perf_counter() - t0:.2f}s: {info}")
    params = torch.tensor(angles, dtype=torch.float64, device=dev)
    out = torch.empty((n_nets, N_SETS, 2), dtype=torch.float64, device=dev)
    obj = torch.empty(N_SETS, dtype=torch.float64, device=dev)
    grad = torch.empty((N_SETS, 2 * P_LAYERS), dtype=torch.float64, device=dev)
    gnet = torch.empty((n_nets, N_SETS, 2 * P_LAYERS), dtype=torch.float64, device=dev)
    st = torch.cuda.Stream()

    # --- accuracy against the closed-form p=1 oracle ---------------------------------
    from oracle import closed_form
    model.batch.grad(params, out=out, obj=obj, grad=grad, grad_net=gnet, stream=st)
    st.synchronize()
    o, ob, gr = out.cpu().numpy(), obj.cpu().numpy(), grad.cpu().numpy()
    err_zz = err_c = err_g = 0.0
    for s in range(N_SETS):
        zz = closed_form.zz_p1(N_VERT, edges, angles[s, 0], angles[s, 1])
        dg, db = closed_form.zz_p1_grad(N_VERT, edges, angles[s, 0], angles[s, 1])
        err_zz = max(err_zz, float(np.max(np.abs(o[:, s, 0] - zz))))
        c_ref = float(np.sum((1 - zz) / 2))
        err_c = max(err_c, abs(ob[s] - c_ref) / max(1.0, abs(c_ref)))
        g_ref = np.array([-0.5 * dg.sum(), -0.5 * db.sum()])
        err_g = max(err_g, float(np.max(np.abs(gr[s] - g_ref)) / max(1.0, np.abs(g_ref).max())))
    log(f"error vs FP64 closed form: zz {err_zz:.2e}  <C> rel {err_c:.2e}  grad rel {err_g:.2e}")

    # plan-time kernel choices (autotuner), outside the timed region
    t0 = time.perf_counter()
    model.batch.autotune(params, reps=10, stream=st)
    st.synchronize()
    info = model.batch.info()
    log(f"autotuned in {time.perf_counter() - t0:.2f}s: {info}")
    if info["sets_per_wave_grad"] > 1:
        kname = f"fused_sets_kernel<float, true, {6 - info['sets_per_wave_grad'] // 2}>"
    else:
        kname = (f"fused_exec_kernel<float, {info['fused_block']}, true, "
                 f"{'true' if info['rec_only'] & 2 else 'false'}, false>")

    # --- timed: fwd+grad steps from the captured graph ----------------------------------
    def replay(with_grad):
        model.batch.run_graph(with_grad, params, obj=obj, grad=grad if with_grad else None, stream=st)

    for _ in range(args.warmup):
        replay(True)
    torch.cuda.synchronize()
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
    log(f"fwd+grad: {ms_step * 1e3:.1f} us/step, {value:.3e} networks/s (wall {wall:.3f}s)")

    # forward only
    for _ in range(args.warmup):
        replay(False)
    ev0.record(st)
    for _ in range(args.steps):
        replay(False)
    ev1.record(st)
    torch.cuda.synchronize()
    ms_fwd = ev0.elapsed_time(ev1) / args.steps
    log(f"fwd: {ms_fwd * 1e3:.1f} us/step")

    # dominant kernel alone (fused executor, adjoint program): HIP events the
    # library records on the launch stream right around each fused launch
    for _ in range(args.warmup):
        model.batch.grad(params, out=out, grad_net=gnet, stream=st)
    model.batch.kernel_timing(True)
    for _ in range(args.steps):
        model.batch.grad(params, out=out, grad_net=gnet, stream=st)
    n_timed, total_ms = model.batch.kernel_time()
    model.batch.kernel_timing(False)
    k_ms = total_ms / max(1, n_timed)
    alg_bytes = (info["bytes_fwd"] + info["bytes_grad"]) * N_SETS
    alg_flops = (info["flops_fwd"] + info["flops_grad"]) * N_SETS
    achieved = alg_bytes / (k_ms * 1e-3)
    log(f"fused kernel: {k_ms * 1e3:.1f} us, {achieved / 1e9:.1f} GB/s algorithmic, "
        f"{alg_flops / (k_ms * 1e-3) / 1e12:.3f} TFLOP/s")

    # plain path: one network per launch, complex64 and complex128 (host sync per network)
    plain = {}
    for name, dt in (("c64", qtn.TN_C64), ("c128", qtn.TN_C128)):
        nets = qaoa.edge_networks(N_VERT, edges, P_LAYERS, dt, order="linegraph", trials=4)
        a0 = angles[0]
        for net in nets:  # plan-time device set-up of every network, outside the timed loops
            net.contract(a0, stream=st)
            net.grad(a0, stream=st)
        t0 = time.perf_counter()
        vals = [net.contract(a0, stream=st) for net in nets]
        dtp = time.perf_counter() - t0
        zz = closed_form.zz_p1(N_VERT, edges, a0[0], a0[1])
        # forward plus adjoint gradient, one network per call (tn_grad)
        t0 = time.perf_counter()
        grads = [net.grad(a0, stream=st) for net in nets]
        dtg = time.perf_counter() - t0
        dg, db = closed_form.zz_p1_grad(N_VERT, edges, a0[0], a0[1])
        gerr = max(float(np.max(np.abs(g - np.array([dg[i], db[i]])))) for i, (_, g) in enumerate(grads))
        plain[name] = {"networks_per_s": len(nets) / dtp,
                       "max_abs_err_zz": float(np.max(np.abs(np.array(vals).real - zz))),
                       "fwd_grad_networks_per_s": len(nets) / dtg, "max_abs_err_grad": gerr}
        log(f"plain {name}: {plain[name]}")

    # dense regime (MFMA path): whole-circuit network of one edge, 6-regular n=20, p=1
    mfma = None
    if not args.no_dense:
        dd, dn = 6, 20
        de = workloads.random_regular_graph(dd, dn, GRAPH_SEED)
        dnet = qaoa.edge_network(dn, de, 1, de[0], dtype=qtn.TN_C64, lightcone=False)
        dnet.set_order(dnet.order_linegraph(trials=8, seed=0))
        dinfo = dnet.plan_info()
        dbatch = qtn.Batch([dnet], max_sets=1)
        dpar = torch.tensor([angles[0]], dtype=torch.float64, device=dev)
        dbatch.autotune(dpar, reps=2, stream=st)
        dout = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
        dbatch.contract(dpar, out=dout, stream=st)
        st.synchronize()
        reps = 5
        ev0.record(st)
        for _ in range(reps):
            dbatch.contract(dpar, out=dout, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        d_ms = ev0.elapsed_time(ev1) / reps
        zz_ref = closed_form.zz_p1(dn, de, angles[0, 0], angles[0, 1])[0]
        # forward + adjoint gradient of the same network (FP32 products)
        dgn = torch.empty((1, 1, 2), dtype=torch.float64, device=dev)
        doutg = torch.empty_like(dout)
        dbatch.grad(dpar, out=doutg, grad_net=dgn, stream=st)
        st.synchronize()
        ev0.record(st)
        for _ in range(reps):
            dbatch.grad(dpar, out=doutg, grad_net=dgn, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        g_ms = ev0.elapsed_time(ev1) / reps
        dbi = dbatch.info()
        g_flops = dbi["flops_fwd"] + dbi["flops_grad"]
        dg_ref, db_ref = closed_form.zz_p1_grad(dn, de, angles[0, 0], angles[0, 1])
        g_err = float(np.max(np.abs(dgn[0, 0].cpu().numpy() - np.array([dg_ref[0], db_ref[0]]))))
        # split-BF16 products on the same network
        dbatch.set_precision(qtn.TN_MFMA_BF16X3)
        dbatch.autotune(dpar, reps=2, stream=st)
        dout2 = torch.empty_like(dout)
        dbatch.contract(dpar, out=dout2, stream=st)
        ev0.record(st)
        for _ in range(reps):
            dbatch.contract(dpar, out=dout2, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        b_ms = ev0.elapsed_time(ev1) / reps
        # complex128: FP64 matrix-core products on the same network
        dnet128 = qaoa.edge_network(dn, de, 1, de[0], dtype=qtn.TN_C128, lightcone=False)
        dnet128.set_order(dnet128.order_linegraph(trials=8, seed=0))
        dbatch128 = qtn.Batch([dnet128], max_sets=1)
        dbatch128.autotune(dpar, reps=2, stream=st)
        dout3 = torch.empty_like(dout)
        dbatch128.contract(dpar, out=dout3, stream=st)
        ev0.record(st)
        for _ in range(reps):
            dbatch128.contract(dpar, out=dout3, stream=st)
        ev1.record(st)
        torch.cuda.synchronize()
        f_ms = ev0.elapsed_time(ev1) / reps
        mfma = {"workload": f"whole-circuit folded network of one edge, QAOA p=1, {dd}-regular n={dn} "
                            f"(no light cone), line-graph order, complex64, 4M FP32 MFMA",
                "peak_bits": dinfo["peak_bits"], "flops_per_pass": dinfo["flops"], "pass_ms": d_ms,
                "tflops": dinfo["flops"] / (d_ms * 1e-3) / 1e12,
                "frac_of_fp32_matrix_peak": dinfo["flops"] / (d_ms * 1e-3) / FP32_MFMA_PEAK,
                "abs_err_zz_vs_closed_form": abs(dout[0, 0, 0].item() - zz_ref),
                "fwd_grad": {"pass_ms": g_ms, "flops_per_pass": g_flops,
                             "tflops": g_flops / (g_ms * 1e-3) / 1e12,
                             "frac_of_fp32_matrix_peak": g_flops / (g_ms * 1e-3) / FP32_MFMA_PEAK,
                             "abs_err_grad_vs_closed_form": g_err},
                "split_bf16": {"pass_ms": b_ms, "tflops_fp32_equivalent": dinfo["flops"] / (b_ms * 1e-3) / 1e12,
                               "abs_err_zz_vs_closed_form": abs(dout2[0, 0, 0].item() - zz_ref)},
                "complex128_fp64": {"pass_ms": f_ms, "tflops": dinfo["flops"] / (f_ms * 1e-3) / 1e12,
                                    "frac_of_fp64_matrix_peak": dinfo["flops"] / (f_ms * 1e-3) / FP64_MFMA_PEAK,
                                    "abs_err_zz_vs_closed_form": abs(dout3[0, 0, 0].item() - zz_ref)}}
        log(f"dense/MFMA: {mfma}")

    nxt = None if args.no_next else next_rows(model, params, edges, st, dev)
    grid = diff = cross = None
    if not args.no_grid:
        # the other configurations run in a child process (its own GPU context): a failure there is
        # recorded in their entries and does not take the headline measurement with it
        import subprocess
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

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        cpu = cpu_baseline(edges, angles)
        log(f"cpu baseline: {cpu}")

    rec = {
        "metric": "QAOA <ZZ> networks contracted/s (fwd+grad)",
        "value": value,
        "unit": "networks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex), fp64 final scalars and gradient sums",
        "data": "synthetic",
        "config": {"workload": f"QAOA Max-Cut p={P_LAYERS}, random {D}-regular graph n={N_VERT} "
                               f"({n_nets} edge light-cone networks) x {N_SETS} angle sets, fwd + adjoint grad, "
                               "line-graph order, one hipGraph replay per step",
                   "networks_per_step": n_nets * N_SETS, "parallelism": "single GPU"},
        "fwd_networks_per_s": n_nets * N_SETS / (ms_fwd * 1e-3),
        "ms_per_step_fwd": ms_fwd,
        "plain_one_network_per_launch": plain,
        "error_vs_fp64_oracle": {"max_abs_zz": err_zz, "max_rel_cost": err_c, "max_rel_grad": err_g},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": traffic_from_profile(kname),
                     "kernel": kname, "kernel_us": k_ms * 1e3, "kernel_launches_timed": n_timed,
                     "algorithmic_bytes_per_launch": alg_bytes, "algorithmic_flops_per_launch": alg_flops},
        "mfma_path": mfma,
        "next_rows": nxt,
        "batching_grid": grid,
        "differentiation_p2_n60": diff,
        "crossover_in_degree": cross,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
