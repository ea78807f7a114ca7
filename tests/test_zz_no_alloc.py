"""The allocation-free batch entry point, tn_batch_grad_noalloc, against
tn_batch_grad on the same batches.

Two calls in a row share the library's static scratch: first a batch split
over the LDS fused, global-arena and level executors (the level networks on
the task executor), then a smaller batch (fewer, smaller networks and fewer
parameter vectors) that runs over what the first left behind. While they run,
the library's allocator is one that records every request and refuses it, so
any device allocation on that path fails the call. Each call's per-network
values, objective and gradients equal tn_batch_grad's on the same batch bit
for bit (same kernels, same order of operations), and the smaller batch
matches the p=1 closed form. A batch whose workspace exceeds the scratch is
refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import closed_form

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _outputs(batch, n_sets):
    z = dict(dtype=torch.float64, device="cuda")
    return (torch.full((batch.n_nets, n_sets, 2), -7.0, **z), torch.full((n_sets,), -7.0, **z),
            torch.full((n_sets, batch.n_params), -7.0, **z),
            torch.full((batch.n_nets, n_sets, batch.n_params), -7.0, **z))


def _noalloc(qtn, batch, params, outs, stream):
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = qtn.lib().tn_batch_grad_noalloc(batch.h, p(params), params.shape[0], *[p(t) for t in outs],
                                         ctypes.c_void_p(stream.cuda_stream))
    if rc != qtn.TN_OK:
        raise qtn.QtnError(rc, qtn.lib().tn_last_error().decode())


def test_noalloc_matches_batch_grad(monkeypatch):
    from paper_1709_03636_amd import qaoa, qtn

    # batch A: 3-regular n=24 p=2 under executor limits that split it three
    # ways; level groups on the task executor
    n_a, e_a = 24, workloads.random_regular_graph(3, 24, 2)
    monkeypatch.setenv("QTN_FUSED_LDS_MAX", "32768")
    monkeypatch.setenv("QTN_GMEM_MAX_MACS", str(1 << 18))
    monkeypatch.setenv("QTN_TASK_MIN", "1")
    monkeypatch.setenv("QTN_GMEM_JOIN", "0")
    model_a = qaoa.MaxCut(n_a, e_a, 2, qtn.TN_C64, order="linegraph", max_sets=4, trials=2)
    for var in ("QTN_FUSED_LDS_MAX", "QTN_GMEM_MAX_MACS", "QTN_TASK_MIN", "QTN_GMEM_JOIN"):
        monkeypatch.delenv(var)
    info = model_a.batch.info()
    assert info["n_fused"] > 0 and info["n_global"] > 0 and info["n_level"] > 0 and info["n_level_tasked"] > 0
    # batch B: 3-regular n=12 p=1, fewer networks and parameter vectors
    n_b, e_b = 12, workloads.random_regular_graph(3, 12, 0)
    model_b = qaoa.MaxCut(n_b, e_b, 1, qtn.TN_C64, order="linegraph", max_sets=2, trials=2)
    ws_a, ws_b = model_a.batch.workspace_bytes(), model_b.batch.workspace_bytes()
    assert ws_b < ws_a <= 64 << 20 and model_b.batch.n_nets < model_a.batch.n_nets
    ang_a = torch.tensor(workloads.qaoa_angles(21, 4, 2), dtype=torch.float64, device="cuda")
    ang_b = torch.tensor(workloads.qaoa_angles(22, 2, 1), dtype=torch.float64, device="cuda")
    outs_a, outs_b = _outputs(model_a.batch, 4), _outputs(model_b.batch, 2)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())

    requests = []

    @qtn._ALLOC_FN
    def refuse(nbytes, ctx):
        requests.append(int(nbytes))
        return None

    @qtn._FREE_FN
    def no_free(ptr, ctx):
        requests.append(-1)

    qtn._device_setup()
    qtn._check(qtn.lib().tn_set_allocator(ctypes.cast(refuse, ctypes.c_void_p), ctypes.cast(no_free, ctypes.c_void_p),
                                          None))
    try:
        _say(f"noalloc call 1: {model_a.batch.n_nets} networks, 4 sets, workspace {ws_a} bytes")
        _noalloc(qtn, model_a.batch, ang_a, outs_a, st)
        _say(f"noalloc call 2: {model_b.batch.n_nets} networks, 2 sets, workspace {ws_b} bytes")
        _noalloc(qtn, model_b.batch, ang_b, outs_b, st)
        st.synchronize()
    finally:
        qtn._check(qtn.lib().tn_set_allocator(ctypes.cast(qtn._alloc_cb, ctypes.c_void_p),
                                              ctypes.cast(qtn._free_cb, ctypes.c_void_p), None))
    assert requests == []
    got_a = [t.cpu().numpy() for t in outs_a]
    got_b = [t.cpu().numpy() for t in outs_b]

    # the allocating entry point on the same batches (workspaces bound here)
    for model, ang, got, tag in ((model_a, ang_a, got_a, "A"), (model_b, ang_b, got_b, "B")):
        ref = _outputs(model.batch, ang.shape[0])
        _say(f"tn_batch_grad reference, batch {tag}")
        model.batch.grad(ang, *ref)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r.cpu().numpy())

    # batch B against the closed form
    for s in range(2):
        g, b = ang_b[s].tolist()
        zz = closed_form.zz_p1(n_b, e_b, g, b)
        dg, db = closed_form.zz_p1_grad(n_b, e_b, g, b)
        assert np.max(np.abs(got_b[0][:, s, 0] - zz)) < 1e-5
        assert np.max(np.abs(got_b[3][:, s, 0] - dg)) < 1e-4 and np.max(np.abs(got_b[3][:, s, 1] - db)) < 1e-4
        assert abs(got_b[1][s] - closed_form.cost_p1(n_b, e_b, g, b)) < 1e-5 * len(e_b)


def test_noalloc_refuses_large_workspace():
    from paper_1709_03636_amd import qaoa, qtn
    e = workloads.random_regular_graph(3, 12, 0)
    model = qaoa.MaxCut(12, e, 1, qtn.TN_C64, order="linegraph", max_sets=1 << 18, trials=2)
    assert model.batch.workspace_bytes() > 64 << 20
    params = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    outs = _outputs(model.batch, 1)
    with pytest.raises(qtn.QtnError, match="static scratch"):
        _noalloc(qtn, model.batch, params, outs, torch.cuda.current_stream())
    assert np.all(outs[1].cpu().numpy() == -7.0)
