"""ctypes binding of the C ABI in include/qtn.h (argument marshalling only).

Every function keeps the C name; the classes Network and Batch wrap the
handles. Device buffers and streams come from PyTorch (torch.cuda tensors and
torch.cuda streams); all compute runs in the library's HIP kernels. There is
no fallback: without the built library every call raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QTN_LIB", os.path.join(HERE, "libqtn.so"))

TN_OK, TN_EINVAL, TN_ENOMEM, TN_EORDER, TN_EDEVICE, TN_ESTATE = 0, -1, -2, -3, -4, -5
TN_H, TN_X, TN_Y, TN_Z, TN_RX, TN_RY, TN_RZ, TN_ZZ, TN_CNOT, TN_CZ, TN_U1, TN_U2, TN_SUPER1, TN_SUPER2, \
    TN_KRAUS1, TN_KRAUS2 = range(16)
TN_AMPLITUDE, TN_PROBABILITY, TN_EXPECTATION = 0, 1, 2
TN_EXEC_FUSED, TN_EXEC_LEVEL, TN_EXEC_GLOBAL = 0, 1, 2
TN_C64, TN_C128 = 0, 1
TN_MFMA_FP32, TN_MFMA_BF16X3, TN_MFMA_FP64 = 1, 2, 3
GATE_KINDS = {"H": TN_H, "X": TN_X, "Y": TN_Y, "Z": TN_Z, "RX": TN_RX, "RY": TN_RY, "RZ": TN_RZ, "ZZ": TN_ZZ,
              "CNOT": TN_CNOT, "CZ": TN_CZ, "U1": TN_U1, "U2": TN_U2, "SUPER1": TN_SUPER1, "SUPER2": TN_SUPER2,
              "KRAUS1": TN_KRAUS1, "KRAUS2": TN_KRAUS2}
ERR_NAMES = {TN_EINVAL: "TN_EINVAL", TN_ENOMEM: "TN_ENOMEM", TN_EORDER: "TN_EORDER", TN_EDEVICE: "TN_EDEVICE",
             TN_ESTATE: "TN_ESTATE"}


class QtnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class tn_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("param", ctypes.c_int32), ("coeff", ctypes.c_double), ("matrix", ctypes.POINTER(ctypes.c_double)),
                ("n_matrices", ctypes.c_int32)]


class tn_target(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("bits", ctypes.POINTER(ctypes.c_uint8)),
                ("pauli", ctypes.POINTER(ctypes.c_uint8)), ("lightcone", ctypes.c_int32),
                ("diagonal", ctypes.c_int32)]


class tn_plan_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_steps", "n_tensors", "n_wires", "peak_bits", "max_rank_wires",
                                               "n_components", "fused", "lds_bytes")] + \
               [(n, ctypes.c_double) for n in ("flops", "bytes", "peak_live_bytes", "grad_bytes")] + \
               [(n, ctypes.c_int32) for n in ("recompute_runs", "reserved")]


class tn_batch_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_nets", "n_fused", "n_level", "n_levels", "lds_bytes_fwd",
                                               "lds_bytes_grad", "n_programs", "fused_block", "rec_only",
                                               "sets_per_wave_fwd", "sets_per_wave_grad", "n_global",
                                               "n_level_groups", "n_level_tasked", "n_level_chunked", "level_launches_fwd",
                                               "level_launches_grad", "level_split_fwd", "level_split_grad")] + \
               [(n, ctypes.c_double) for n in ("flops_fwd", "bytes_fwd", "flops_grad", "bytes_grad")] + \
               [("exec_flops", ctypes.c_double * 3), ("exec_bytes", ctypes.c_double * 3),
                ("level_mfma_flops", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "tn_build": (_I, [ctypes.POINTER(tn_gate), _I, _I, _PD, ctypes.POINTER(tn_target), _I, _I, ctypes.POINTER(_P)]),
    "tn_wires": (_I, [_P, _PI, _PI, _PI]),
    "tn_order_stochastic": (_I, [_P, ctypes.c_uint64, _I, _PI]),
    "tn_order_linegraph": (_I, [_P, _I, _D, ctypes.c_uint64, _PI]),
    "tn_set_order": (_I, [_P, _PI, _I]),
    "tn_set_memory_limit": (_I, [_P, ctypes.c_uint64]),
    "tn_plan_info": (_I, [_P, ctypes.POINTER(tn_plan_stats)]),
    "tn_plan_steps": (_I, [_P, _PI]),
    "tn_contract": (_I, [_P, _PD, _PD, _P]),
    "tn_grad": (_I, [_P, _PD, _PD, _PD, _P]),
    "tn_batch_create": (_I, [ctypes.POINTER(_P), _I, _PD, _D, _I, ctypes.POINTER(_P)]),
    "tn_batch_workspace_bytes": (_I, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "tn_batch_set_workspace": (_I, [_P, _P, ctypes.c_int64]),
    "tn_set_allocator": (_I, [_P, _P, _P]),
    "tn_batch_contract": (_I, [_P, _P, _I, _P, _P, _P]),
    "tn_batch_grad": (_I, [_P, _P, _I, _P, _P, _P, _P, _P]),
    "tn_batch_grad_noalloc": (_I, [_P, _P, _I, _P, _P, _P, _P, _P]),
    "tn_batch_run_graph": (_I, [_P, _I, _P, _I, _P, _P, _P, _P, _P]),
    "tn_batch_info": (_I, [_P, ctypes.POINTER(tn_batch_stats)]),
    "tn_batch_autotune": (_I, [_P, _P, _I, _I, ctypes.c_char_p, _P]),
    "tn_batch_apply_tuning": (_I, [_P, ctypes.c_char_p]),
    "tn_batch_set_precision": (_I, [_P, _I]),
    "tn_batch_kernel_timing": (_I, [_P, _I]),
    "tn_batch_kernel_time": (_I, [_P, _I, _PI, _PD]),
    "tn_contract_batch": (_I, [ctypes.POINTER(_P), _I, _P, _I, _P, _P]),
    "tn_grad_batch": (_I, [ctypes.POINTER(_P), _I, _P, _I, _P, _P, _P]),
    "tn_bind_params": (_I, [_P, _P, _I, _P, ctypes.POINTER(ctypes.c_int64), _P]),
    "tn_sv_workspace_bytes": (ctypes.c_int64, [_I]),
    "tn_sv_maxcut_p1": (_I, [_I, _PI, _I, _D, _D, _P, ctypes.c_int64, _P, _P]),
    "tn_free": (None, [_P]),
    "tn_batch_free": (None, [_P]),
    "tn_last_error": (ctypes.c_char_p, []),
    "tn_version": (ctypes.c_char_p, []),
}


def lib():
    """Load libqtn.so (built in-tree by build_lib); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1709_03636_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != TN_OK:
        raise QtnError(rc, lib().tn_last_error().decode())


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# Device memory the library needs beyond a batch's bound workspace (the
# one-network path, batches run without a workspace, autotuner scratch) comes
# from PyTorch's allocator through tn_set_allocator.
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_torch_blocks = {}


def _torch_alloc(nbytes, ctx):
    import torch
    t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    _torch_blocks[t.data_ptr()] = t
    return t.data_ptr()


def _torch_free(ptr, ctx):
    _torch_blocks.pop(ptr, None)


_alloc_cb = _ALLOC_FN(_torch_alloc)
_free_cb = _FREE_FN(_torch_free)
_allocator_set = False


def _device_setup():
    """Route the library's device allocations through PyTorch (once)."""
    global _allocator_set
    if not _allocator_set:
        _check(lib().tn_set_allocator(ctypes.cast(_alloc_cb, _P), ctypes.cast(_free_cb, _P), None))
        _allocator_set = True


def _stream(stream):
    _device_setup()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def sv_maxcut_p1(n, edges, gamma, beta, workspace=None, stream=None):
    """<C> of the p=1 QAOA Max-Cut state from a full 2^n complex64 state vector
    on the GPU (tn_sv_maxcut_p1; the Hilbert-space comparator, not the
    tensor-network path). workspace: optional cuda uint8 tensor of at least
    tn_sv_workspace_bytes(n) bytes, reused across calls. Returns a float."""
    import torch
    need = lib().tn_sv_workspace_bytes(n)
    if need < 0:
        raise QtnError(TN_EINVAL, f"no state-vector workspace for {n} qubits")
    st = stream if stream is not None else torch.cuda.current_stream()
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    st.wait_stream(torch.cuda.current_stream())  # the buffers exist before the launch stream uses them
    _check(lib().tn_sv_maxcut_p1(n, e.ctypes.data_as(_PI), len(e) // 2, float(gamma), float(beta),
                                 _dptr(workspace), workspace.numel(), _dptr(out), _stream(st)))
    st.synchronize()  # the result is final before `out` can be freed or read
    return float(out.item())


def make_gates(gates):
    """Gate tuples (kind, q0, q1, param, coeff[, matrix]) -> tn_gate array (+ keep-alive list). For
    KRAUS1 / KRAUS2 the matrix entry is the list of Kraus operators (folded by tn_build)."""
    arr = (tn_gate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        kind, q0, q1, param, coeff = g[:5]
        mat = g[5] if len(g) > 5 else None
        k = GATE_KINDS[kind] if isinstance(kind, str) else int(kind)
        mp, nm = None, 0
        if mat is not None:
            a = np.asarray(mat, dtype=np.complex128)
            if k in (TN_KRAUS1, TN_KRAUS2):
                d = 2 if k == TN_KRAUS1 else 4
                a = a.reshape(-1, d, d)
                nm = a.shape[0]
            m = np.ascontiguousarray(a.ravel().view(np.float64))
            keep.append(m)
            mp = m.ctypes.data_as(_PD)
        arr[i] = tn_gate(k, q0, q1, param, coeff, mp, nm)
    return arr, keep


class Network:
    """A built network (tn_build) with an optional order (tn_set_order)."""

    def __init__(self, n_qubits, gates, mode, target, n_params=0, init=None, dtype=TN_C64, lightcone=True,
                 diagonal=False):
        garr, keep = make_gates(gates)
        tv = np.ascontiguousarray(np.asarray(target, dtype=np.uint8))
        t = tn_target(mode, None, None, 1 if lightcone else 0, 1 if diagonal else 0)
        if mode == TN_EXPECTATION:
            t.pauli = tv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        else:
            t.bits = tv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        ip = None
        if init is not None:
            iv = np.ascontiguousarray(np.asarray(init, dtype=np.complex128).reshape(n_qubits, 2).view(np.float64))
            keep.append(iv)
            ip = iv.ctypes.data_as(_PD)
        h = _P()
        _check(lib().tn_build(garr, len(gates), n_qubits, ip, ctypes.byref(t), n_params, dtype, ctypes.byref(h)))
        self.h = h
        self.n_params = n_params
        self.dtype = dtype

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_free(self.h)
            self.h = None

    def wires(self):
        nw, nt = _I(), _I()
        _check(lib().tn_wires(self.h, ctypes.byref(nw), ctypes.byref(nt), None))
        ends = np.zeros(2 * nw.value, dtype=np.int32)
        _check(lib().tn_wires(self.h, ctypes.byref(nw), ctypes.byref(nt), ends.ctypes.data_as(_PI)))
        return nw.value, nt.value, ends.reshape(-1, 2)

    @property
    def n_wires(self):
        return self.wires()[0]

    def order_stochastic(self, seed=0, max_rej=0):
        pi = np.zeros(self.n_wires, dtype=np.int32)
        _check(lib().tn_order_stochastic(self.h, seed, max_rej, pi.ctypes.data_as(_PI)))
        return pi

    def order_linegraph(self, trials=8, budget_s=0.0, seed=0):
        pi = np.zeros(self.n_wires, dtype=np.int32)
        _check(lib().tn_order_linegraph(self.h, trials, budget_s, seed, pi.ctypes.data_as(_PI)))
        return pi

    def set_order(self, pi):
        pi = np.ascontiguousarray(np.asarray(pi, dtype=np.int32))
        _check(lib().tn_set_order(self.h, pi.ctypes.data_as(_PI), len(pi)))

    def set_memory_limit(self, nbytes):
        _check(lib().tn_set_memory_limit(self.h, int(nbytes)))

    def plan_info(self):
        s = tn_plan_stats()
        _check(lib().tn_plan_info(self.h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in s._fields_}

    def plan_steps(self):
        n = self.plan_info()["n_steps"]
        d = np.zeros(3 * max(1, n), dtype=np.int32)
        _check(lib().tn_plan_steps(self.h, d.ctypes.data_as(_PI)))
        return d[:3 * n].reshape(-1, 3)

    def contract(self, params=(), stream=None):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        out = np.zeros(2)
        _check(lib().tn_contract(self.h, p.ctypes.data_as(_PD) if p.size else None, out.ctypes.data_as(_PD),
                                 _stream(stream)))
        return complex(out[0], out[1])

    def grad(self, params, stream=None):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        g = np.zeros(max(1, self.n_params))
        v = ctypes.c_double()
        _check(lib().tn_grad(self.h, p.ctypes.data_as(_PD) if p.size else None, ctypes.byref(v),
                             g.ctypes.data_as(_PD), _stream(stream)))
        return v.value, g[:self.n_params]

    def bind_params(self, params_dev, n_sets, out_dev=None, stream=None):
        per = ctypes.c_int64()
        _check(lib().tn_bind_params(self.h, None, 0, None, ctypes.byref(per), None))
        if out_dev is None:
            return per.value
        _check(lib().tn_bind_params(self.h, _dptr(params_dev), n_sets, _dptr(out_dev), ctypes.byref(per),
                                    _stream(stream)))
        return per.value


class Batch:
    """Many networks x many parameter vectors (tn_batch_*). The device
    workspace is a torch uint8 tensor bound on first use (or explicitly by
    bind_workspace); device tensors passed to the calls are checked for dtype,
    device, layout and size before anything is launched."""

    def __init__(self, nets, coef=None, offset=0.0, max_sets=1):
        self.nets = list(nets)
        arr = (_P * len(self.nets))(*[n.h for n in self.nets])
        cp = None
        if coef is not None:
            self._coef = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
            cp = self._coef.ctypes.data_as(_PD)
        h = _P()
        _check(lib().tn_batch_create(arr, len(self.nets), cp, float(offset), max_sets, ctypes.byref(h)))
        self.h = h
        self.max_sets = max_sets
        self.n_params = self.nets[0].n_params
        self.n_nets = len(self.nets)
        self.workspace = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tn_batch_free(self.h)
            self.h = None

    def workspace_bytes(self):
        n = ctypes.c_int64()
        _check(lib().tn_batch_workspace_bytes(self.h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, workspace=None):
        """Bind a cuda uint8 tensor (allocated here when None) as the batch's
        device workspace (tn_batch_set_workspace)."""
        import torch
        need = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
        if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous() \
                or workspace.numel() < need:
            raise QtnError(TN_EINVAL, f"workspace must be a contiguous cuda uint8 tensor of at least {need} bytes")
        _device_setup()
        _check(lib().tn_batch_set_workspace(self.h, _dptr(workspace), workspace.numel()))
        self.workspace = workspace

    def _ready(self):
        if self.workspace is None:
            self.bind_workspace()

    def _n_sets(self, params):
        """Check params (cuda float64 [n_sets, n_params], contiguous) and return n_sets."""
        if params.dim() != 2 or params.shape[1] != self.n_params:
            raise QtnError(TN_EINVAL, f"params must be [n_sets, {self.n_params}], got {tuple(params.shape)}")
        _need_f64(params, "params", params.numel())
        n = params.shape[0]
        if not 1 <= n <= self.max_sets:
            raise QtnError(TN_EINVAL, f"n_sets {n} outside 1..{self.max_sets}")
        return n

    def _outs(self, n, out=None, obj=None, grad=None, grad_net=None):
        _need_f64(out, "out", self.n_nets * n * 2)
        _need_f64(obj, "obj", n)
        _need_f64(grad, "grad", n * self.n_params)
        _need_f64(grad_net, "grad_net", self.n_nets * n * self.n_params)

    def info(self):
        s = tn_batch_stats()
        _check(lib().tn_batch_info(self.h, ctypes.byref(s)))
        return {n: (list(getattr(s, n)) if n.startswith("exec_") else getattr(s, n)) for n, _ in s._fields_}

    def autotune(self, params, reps=3, cache_path=None, stream=None):
        """Pick fused workgroup size and MFMA/thin per large-op shape (tn_batch_autotune)."""
        n = self._n_sets(params)
        self._ready()
        cp = cache_path.encode() if cache_path else None
        _check(lib().tn_batch_autotune(self.h, _dptr(params), n, reps, cp, _stream(stream)))

    def set_precision(self, mfma_precision):
        """TN_MFMA_FP32 or TN_MFMA_BF16X3 (complex64 batch), TN_MFMA_FP64 (complex128 batch)."""
        _check(lib().tn_batch_set_precision(self.h, mfma_precision))

    def kernel_timing(self, enable=True):
        """Record HIP events around later eager executor launches (tn_batch_kernel_timing)."""
        _check(lib().tn_batch_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self, executor=0):
        """(launches timed, summed milliseconds) of one executor (TN_EXEC_FUSED, TN_EXEC_LEVEL,
        TN_EXEC_GLOBAL) since the last call for it (tn_batch_kernel_time)."""
        n, ms = ctypes.c_int32(), ctypes.c_double()
        _check(lib().tn_batch_kernel_time(self.h, executor, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def apply_tuning(self, cache_path):
        _check(lib().tn_batch_apply_tuning(self.h, cache_path.encode()))

    def contract(self, params, out=None, obj=None, stream=None):
        """params: cuda float64 [n_sets, n_params]; out: [n_nets, n_sets, 2]; obj: [n_sets]."""
        n = self._n_sets(params)
        self._outs(n, out, obj)
        self._ready()
        _check(lib().tn_batch_contract(self.h, _dptr(params), n, _dptr(out), _dptr(obj), _stream(stream)))

    def grad(self, params, out=None, obj=None, grad=None, grad_net=None, stream=None):
        """As contract, plus grad: [n_sets, n_params], grad_net: [n_nets, n_sets, n_params]."""
        n = self._n_sets(params)
        self._outs(n, out, obj, grad, grad_net)
        self._ready()
        _check(lib().tn_batch_grad(self.h, _dptr(params), n, _dptr(out), _dptr(obj), _dptr(grad),
                                   _dptr(grad_net), _stream(stream)))

    def run_graph(self, with_grad, params, out=None, obj=None, grad=None, grad_net=None, stream=None):
        n = self._n_sets(params)
        self._outs(n, out, obj, grad if with_grad else None, grad_net if with_grad else None)
        self._ready()
        _check(lib().tn_batch_run_graph(self.h, 1 if with_grad else 0, _dptr(params), n, _dptr(out),
                                        _dptr(obj), _dptr(grad), _dptr(grad_net), _stream(stream)))


def _need_f64(t, name, numel):
    """A device output or input: None, or a contiguous cuda float64 tensor of
    at least `numel` entries."""
    if t is None:
        return
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() < numel:
        raise QtnError(TN_EINVAL, f"{name} must be a contiguous cuda float64 tensor of at least {numel} entries "
                                  f"(got {t.dtype}, {'cuda' if t.is_cuda else 'cpu'}, "
                                  f"{'contiguous' if t.is_contiguous() else 'strided'}, {t.numel()})")
