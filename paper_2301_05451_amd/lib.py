"""ctypes binding of ``libtq.so`` (argument marshalling only; every step runs in HIP kernels).

Raises at import if the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
# TQ_LIBRARY selects another build of the same library (e.g. the host-sanitizer build)
LIB_PATH = os.environ.get("TQ_LIBRARY") or os.path.join(_HERE, "libtq.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2301_05451_amd.build`")
_lib = ct.CDLL(LIB_PATH)

HIP_BUILD_VERSION = _lib.tq_hip_build_version()
HIP_RUNTIME_VERSION = _lib.tq_hip_runtime_version()


def _major_minor(v):
    return (v // 10000000, (v // 100000) % 100) if v >= 0 else (-1, -1)


if _major_minor(HIP_RUNTIME_VERSION) < _major_minor(HIP_BUILD_VERSION):
    raise ImportError(
        f"libtq.so was built for HIP {HIP_BUILD_VERSION} but is bound to an older HIP runtime "
        f"{HIP_RUNTIME_VERSION} (torch's bundled one): import paper_2301_05451_amd before torch")

TQ_C64, TQ_C128 = 0, 1
STATUS = {0: "TQ_OK", 1: "TQ_EINVAL", 2: "TQ_ESIZE", 3: "TQ_ENOTSUP", 4: "TQ_EHIP", 5: "TQ_EWORKSPACE", 6: "TQ_ENOMEM"}


class TQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Batch(ct.Structure):
    _fields_ = [("count", ct.c_int32), ("n_qubits", ct.c_void_p), ("gate_off", ct.c_void_p),
                ("n_gates", ct.c_void_p), ("param_off", ct.c_void_p), ("state_off", ct.c_void_p)]


class SvOpts(ct.Structure):
    _fields_ = [("mode", ct.c_int32), ("tile_bits", ct.c_int32), ("reg_bits", ct.c_int32), ("coal_bits", ct.c_int32)]


_vp = ct.c_void_p
_i32 = ct.c_int32
_lib.tq_last_error.restype = ct.c_char_p
_lib.tq_version.restype = ct.c_int
_lib.tq_ctx_create.argtypes = [ct.c_int, ct.POINTER(_vp)]
_lib.tq_ctx_create.restype = ct.c_int
_lib.tq_ctx_destroy.argtypes = [_vp]
_lib.tq_ctx_destroy.restype = None
_lib.tq_sv_apply.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, _vp, ct.POINTER(SvOpts), _vp]
_lib.tq_sv_apply.restype = ct.c_int
_lib.tq_expval.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _i32, _i32, _vp, _vp]
_lib.tq_expval.restype = ct.c_int
_lib.tq_sv_init.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), ct.c_int64, _vp, _vp]
_lib.tq_sv_init.restype = ct.c_int
_lib.tq_sv_plan_info.argtypes = [_vp, ct.c_int, _i32, _vp, _i32, ct.POINTER(SvOpts), ct.POINTER(ct.c_int64)]
_lib.tq_sv_plan_info.restype = ct.c_int
_lib.tq_sv_backward_workspace.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, _i32, _i32,
                                          ct.POINTER(SvOpts)]
_lib.tq_sv_backward_workspace.restype = ct.c_int64
_lib.tq_sv_backward.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp,
                                _vp, ct.POINTER(SvOpts), _vp, ct.c_int64, _vp]
_lib.tq_sv_backward.restype = ct.c_int


def raw():
    """The loaded ctypes library (for tests that call the C ABI directly)."""
    return _lib


def check(status):
    if status != 0:
        raise TQError(status, _lib.tq_last_error().decode())


def last_error():
    return _lib.tq_last_error().decode()


class Context:
    def __init__(self, device=0):
        h = _vp()
        check(_lib.tq_ctx_create(int(device), ct.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            _lib.tq_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctx = {}


def context(device=None):
    import torch
    if device is None:
        device = torch.cuda.current_device()
    if device not in _ctx:
        _ctx[device] = Context(device)
    return _ctx[device]


class BatchSpec:
    """Host arrays of a tq_batch plus the concatenated gate list and per-circuit sizes."""

    def __init__(self, n_qubits, gate_off, n_gates, param_off, state_off, n_params, gates):
        self.n_qubits = np.ascontiguousarray(n_qubits, dtype=np.int32)
        self.gate_off = np.ascontiguousarray(gate_off, dtype=np.int64)
        self.n_gates = np.ascontiguousarray(n_gates, dtype=np.int32)
        self.param_off = np.ascontiguousarray(param_off, dtype=np.int64)
        self.state_off = np.ascontiguousarray(state_off, dtype=np.int64)
        self.n_params = np.ascontiguousarray(n_params, dtype=np.int32)
        self.gates = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
        self.count = int(self.n_qubits.shape[0])
        self.total_amps = int(max((self.state_off + (1 << self.n_qubits.astype(np.int64))).max(), 0)) if self.count else 0
        self.total_params = int((self.param_off + self.n_params).max()) if self.count else 0
        self._c = Batch(self.count, self.n_qubits.ctypes.data, self.gate_off.ctypes.data, self.n_gates.ctypes.data,
                        self.param_off.ctypes.data, self.state_off.ctypes.data)

    @property
    def c(self):
        return self._c

    @staticmethod
    def uniform(n, gates, count, n_params):
        """``count`` circuits sharing one gate list; params [count, n_params], states [count, 2^n]."""
        g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
        return BatchSpec(np.full(count, n), np.zeros(count), np.full(count, g.shape[0]),
                         np.arange(count) * n_params, np.arange(count) * (1 << n), np.full(count, n_params), g)

    @staticmethod
    def from_circuits(circs):
        """Circuits of different structure packed one after another."""
        gates, goff, poff, soff = [], [], [], []
        go = po = so = 0
        for c in circs:
            goff.append(go); poff.append(po); soff.append(so)
            gates.append(c.gates)
            go += c.gates.shape[0]; po += c.n_params; so += 1 << c.n
        g = np.concatenate(gates) if gates else np.zeros(0, dtype=W.GATE_DTYPE)
        return BatchSpec([c.n for c in circs], goff, [c.gates.shape[0] for c in circs], poff, soff,
                         [c.n_params for c in circs], g)


def _dt(states):
    import torch
    if states.dtype == torch.complex64:
        return TQ_C64
    if states.dtype == torch.complex128:
        return TQ_C128
    raise TypeError("states must be complex64 or complex128")


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _opts(mode=0, tile_bits=0, reg_bits=0, coal_bits=0):
    return SvOpts(int(mode), int(tile_bits), int(reg_bits), int(coal_bits))


def _check_tensors(states, params, spec):
    import torch
    if not states.is_cuda or not states.is_contiguous():
        raise ValueError("states must be a contiguous CUDA tensor")
    if states.numel() < spec.total_amps:
        raise ValueError(f"states has {states.numel()} amplitudes, batch needs {spec.total_amps}")
    want = torch.float32 if states.dtype == torch.complex64 else torch.float64
    if params is not None:
        if params.dtype != want or not params.is_cuda or not params.is_contiguous():
            raise ValueError(f"params must be a contiguous CUDA {want} tensor")
        if params.numel() < spec.total_params:
            raise ValueError("params tensor too small for the batch")


def sv_apply(states, params, spec: BatchSpec, mode=0, tile_bits=0, reg_bits=0, coal_bits=0, ctx=None):
    """In-place |psi_i> <- U_i |psi_i> for every circuit of ``spec`` (tq_sv_apply)."""
    _check_tensors(states, params, spec)
    ctx = ctx or context(states.device.index)
    o = _opts(mode, tile_bits, reg_bits, coal_bits)
    check(_lib.tq_sv_apply(ctx.h, _dt(states), ct.byref(spec.c), spec.gates.ctypes.data, spec.n_params.ctypes.data,
                           params.data_ptr(), states.data_ptr(), ct.byref(o), _stream()))
    return states


_lib.tq_sv_run.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, ct.c_int64, _vp, ct.POINTER(SvOpts), _vp]
_lib.tq_sv_run.restype = ct.c_int


def sv_run(states, params, spec: BatchSpec, basis=0, mode=0, tile_bits=0, reg_bits=0, coal_bits=0, ctx=None):
    """|psi_i> <- U_i |basis> for every circuit of ``spec`` (tq_sv_run): the states' contents
    are not read; in fused mode the first stage forms the basis state itself."""
    _check_tensors(states, params, spec)
    ctx = ctx or context(states.device.index)
    o = _opts(mode, tile_bits, reg_bits, coal_bits)
    check(_lib.tq_sv_run(ctx.h, _dt(states), ct.byref(spec.c), spec.gates.ctypes.data, spec.n_params.ctypes.data,
                         params.data_ptr(), ct.c_int64(basis), states.data_ptr(), ct.byref(o), _stream()))
    return states


PLAN_FIELDS = ("sweeps", "ops", "phases", "exchanges", "tile_bits", "reg_bits", "flops_per_amp", "mats")


def plan_info(n, gates, dtype_c128=False, mode=0, tile_bits=0, reg_bits=0, coal_bits=0, ctx=None, host=False):
    """Schedule shape for one circuit structure (tq_sv_plan_info), as a dict. mode 0 fused,
    1 plain, 2 the reverse sweep of the adjoint; ``host`` builds it without a context (no
    device needed)."""
    h = None if host else (ctx or context()).h
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    out = (ct.c_int64 * 8)()
    o = _opts(mode, tile_bits, reg_bits, coal_bits)
    check(_lib.tq_sv_plan_info(h, TQ_C128 if dtype_c128 else TQ_C64, int(n), g.ctypes.data, int(g.shape[0]),
                               ct.byref(o), out))
    return dict(zip(PLAN_FIELDS, [int(v) for v in out]))


def expval(states, spec: BatchSpec, terms, n_obs, ctx=None):
    """[count, n_obs] real expectation values of Z-string sums (tq_expval)."""
    import torch
    _check_tensors(states, None, spec)
    ctx = ctx or context(states.device.index)
    terms = np.ascontiguousarray(terms, dtype=W.ZTERM_DTYPE)
    rdt = torch.float32 if states.dtype == torch.complex64 else torch.float64
    out = torch.empty((spec.count, n_obs), dtype=rdt, device=states.device)
    check(_lib.tq_expval(ctx.h, _dt(states), ct.byref(spec.c), states.data_ptr(), terms.ctypes.data,
                         int(terms.shape[0]), int(n_obs), out.data_ptr(), _stream()))
    return out


_lib.tq_expval_pauli.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _i32, _i32, _vp, _vp]
_lib.tq_expval_pauli.restype = ct.c_int
_lib.tq_probs.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _i32, _vp, _vp]
_lib.tq_probs.restype = ct.c_int
_lib.tq_lower_gates.argtypes = [_vp, _i32, _vp, _i32]
_lib.tq_lower_gates.restype = ct.c_int32


def expval_pauli(states, spec: BatchSpec, terms, n_obs, ctx=None):
    """[count, n_obs] expectation values of Pauli-string sums (tq_expval_pauli)."""
    import torch
    _check_tensors(states, None, spec)
    ctx = ctx or context(states.device.index)
    terms = np.ascontiguousarray(terms, dtype=W.PAULI_DTYPE)
    rdt = torch.float32 if states.dtype == torch.complex64 else torch.float64
    out = torch.empty((spec.count, n_obs), dtype=rdt, device=states.device)
    check(_lib.tq_expval_pauli(ctx.h, _dt(states), ct.byref(spec.c), states.data_ptr(), terms.ctypes.data,
                               int(terms.shape[0]), int(n_obs), out.data_ptr(), _stream()))
    return out


def probs(states, spec: BatchSpec, qubits, ctx=None):
    """[count, 2^len(qubits)] marginal probabilities of the listed qubits (tq_probs)."""
    import torch
    _check_tensors(states, None, spec)
    ctx = ctx or context(states.device.index)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    rdt = torch.float32 if states.dtype == torch.complex64 else torch.float64
    out = torch.empty((spec.count, 1 << len(q)), dtype=rdt, device=states.device)
    check(_lib.tq_probs(ctx.h, _dt(states), ct.byref(spec.c), states.data_ptr(), q.ctypes.data, int(q.shape[0]),
                        out.data_ptr(), _stream()))
    return out


_lib.tq_optimizer_step.argtypes = [ct.c_int, _i32, _vp, _vp, _vp, _vp, _i32, ct.c_double, ct.c_double, ct.c_double,
                                   ct.c_double, ct.c_int64, _vp]
_lib.tq_optimizer_step.restype = ct.c_int


def optimizer_step(params, grad, lr, step=1, m=None, v=None, adam=False, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place update of params (tq_optimizer_step): gradient descent, or Adam with moments m, v."""
    import torch
    dt = TQ_C128 if params.dtype == torch.float64 else TQ_C64
    check(_lib.tq_optimizer_step(dt, 1 if adam else 0, params.data_ptr(), grad.data_ptr(),
                                 m.data_ptr() if m is not None else None, v.data_ptr() if v is not None else None,
                                 int(step), float(lr), float(beta1), float(beta2), float(eps),
                                 ct.c_int64(params.numel()), _stream()))
    return params


_lib.tq_peak_probe.argtypes = [_i32, _vp, ct.c_uint64, _i32, ct.POINTER(ct.c_double), _vp]
_lib.tq_peak_probe.restype = ct.c_int

PEAK_COPY, PEAK_FP32_FMA, PEAK_FP32_MFMA, PEAK_FP64_MFMA, PEAK_READ = 0, 1, 2, 3, 4


def peak_probe(kind, buf, iters=1):
    """Enqueue one attainable-peak probe launch (tq_peak_probe) on the current stream over the
    device tensor buf; returns the work it does (bytes for PEAK_COPY and PEAK_READ, flops otherwise)."""
    w = ct.c_double(0.0)
    check(_lib.tq_peak_probe(int(kind), buf.data_ptr(), ct.c_uint64(buf.numel() * buf.element_size()), int(iters),
                             ct.byref(w), _stream()))
    return w.value


_lib.tq_ctx_export_tuning.argtypes = [_vp, _vp, ct.c_int64]
_lib.tq_ctx_export_tuning.restype = ct.c_int64
_lib.tq_ctx_import_tuning.argtypes = [_vp, _vp, ct.c_int64]
_lib.tq_ctx_import_tuning.restype = ct.c_int


def export_tuning(ctx=None) -> bytes:
    """The context's autotune table as bytes (tq_ctx_export_tuning)."""
    ctx = ctx or context()
    n = _lib.tq_ctx_export_tuning(ctx.h, None, 0)
    if n < 0:
        raise TQError(1, last_error())
    buf = ct.create_string_buffer(int(n))
    if _lib.tq_ctx_export_tuning(ctx.h, buf, n) != n:
        raise TQError(2, last_error())
    return buf.raw


def import_tuning(data: bytes, ctx=None):
    """Load an autotune table written by export_tuning into the context (tq_ctx_import_tuning)."""
    ctx = ctx or context()
    buf = ct.create_string_buffer(bytes(data), len(data))
    check(_lib.tq_ctx_import_tuning(ctx.h, buf, len(data)))


def save_tuning(path, ctx=None):
    with open(path, "wb") as f:
        f.write(export_tuning(ctx))


def load_tuning(path, ctx=None):
    with open(path, "rb") as f:
        import_tuning(f.read(), ctx)


_lib.tq_pauli_decompose.argtypes = [_vp, _i32, _vp, ct.c_double, _i32, _vp, _i32]
_lib.tq_pauli_decompose.restype = ct.c_int32


def pauli_decompose(herm, qubits, obs=0, tol=1e-14):
    """Pauli terms of a Hermitian matrix on ``qubits`` (tq_pauli_decompose)."""
    h = np.ascontiguousarray(np.asarray(herm, dtype=np.complex128)).view(np.float64)
    q = np.ascontiguousarray(qubits, dtype=np.int32)
    n = _lib.tq_pauli_decompose(h.ctypes.data, int(q.shape[0]), q.ctypes.data, float(tol), int(obs), None, 0)
    if n < 0:
        raise TQError(1, last_error())
    out = np.zeros(n, dtype=W.PAULI_DTYPE)
    if n:
        check(0 if _lib.tq_pauli_decompose(h.ctypes.data, int(q.shape[0]), q.ctypes.data, float(tol), int(obs),
                                           out.ctypes.data, n) == n else 1)
    return out


def expval_hermitian(states, spec: BatchSpec, herm, qubits, ctx=None):
    """[count] <psi|H|psi> for a Hermitian matrix H on the listed qubits (decomposition +
    tq_expval_pauli)."""
    return expval_pauli(states, spec, pauli_decompose(herm, qubits), 1, ctx)[:, 0]


def lower_gates(gates):
    """The gate list as the kernels apply it (tq_lower_gates: controlled rotations lowered)."""
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    n = _lib.tq_lower_gates(g.ctypes.data, int(g.shape[0]), None, 0)
    if n < 0:
        raise TQError(1, last_error())
    out = np.zeros(n, dtype=W.GATE_DTYPE)
    check(0 if _lib.tq_lower_gates(g.ctypes.data, int(g.shape[0]), out.ctypes.data, n) == n else 1)
    return out


_lib.tq_expval_noalloc.argtypes = [ct.c_int, _i32, _i32, ct.c_int64, _vp, _vp, _i32, _i32, _vp, _vp]
_lib.tq_expval_noalloc.restype = ct.c_int


def expval_noalloc(states, n, count, terms, n_obs, out, stride=None):
    """tq_expval_noalloc into the caller's ``out`` [count, n_obs] (the call allocates nothing)."""
    terms = np.ascontiguousarray(terms, dtype=W.ZTERM_DTYPE)
    stride = (1 << n) if stride is None else int(stride)
    check(_lib.tq_expval_noalloc(_dt(states), int(n), int(count), ct.c_int64(stride), states.data_ptr(),
                                 terms.ctypes.data, int(terms.shape[0]), int(n_obs), out.data_ptr(), _stream()))
    return out


def sv_backward(states, params, spec: BatchSpec, terms, n_obs, grad_out, mode=0, tile_bits=0, reg_bits=0, ctx=None,
                work=None):
    """Adjoint gradients d(sum grad_out * <O>)/d params, same layout as params (tq_sv_backward).
    ``work`` (optional uint8 CUDA tensor) is the caller workspace; a new one is taken from the
    torch allocator when it is missing or too small."""
    import torch
    _check_tensors(states, params, spec)
    ctx = ctx or context(states.device.index)
    terms = np.ascontiguousarray(terms, dtype=W.ZTERM_DTYPE)
    grad_out = grad_out.to(device=params.device, dtype=params.dtype).contiguous()
    if grad_out.numel() < spec.count * n_obs:
        raise ValueError(f"grad_out needs {spec.count} x {n_obs} entries")
    grad = torch.empty_like(params)
    o = _opts(mode, tile_bits, reg_bits, 0)
    need = sv_backward_workspace(states, spec, terms, n_obs, mode, tile_bits, reg_bits, ctx)
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device=states.device)
    check(_lib.tq_sv_backward(ctx.h, _dt(states), ct.byref(spec.c), spec.gates.ctypes.data,
                              spec.n_params.ctypes.data, params.data_ptr(), states.data_ptr(), terms.ctypes.data,
                              int(terms.shape[0]), int(n_obs), grad_out.data_ptr(), grad.data_ptr(), ct.byref(o),
                              work.data_ptr(), ct.c_int64(work.numel()), _stream()))
    return grad


_lib.tq_sv_backward_pauli.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp,
                                      _vp, ct.POINTER(SvOpts), _vp, ct.c_int64, _vp]
_lib.tq_sv_backward_pauli.restype = ct.c_int


def sv_backward_pauli(states, params, spec: BatchSpec, pauli_terms, n_obs, grad_out, tile_bits=0, reg_bits=0,
                      ctx=None):
    """Adjoint gradients for Pauli-string observables (tq_sv_backward_pauli)."""
    import torch
    _check_tensors(states, params, spec)
    ctx = ctx or context(states.device.index)
    pt = np.ascontiguousarray(pauli_terms, dtype=W.PAULI_DTYPE)
    grad_out = grad_out.to(device=params.device, dtype=params.dtype).contiguous()
    grad = torch.empty_like(params)
    o = _opts(0, tile_bits, reg_bits, 0)
    need = sv_backward_workspace(states, spec, W.zterms([]), n_obs, 0, tile_bits, reg_bits, ctx)
    work = torch.empty(need, dtype=torch.uint8, device=states.device)
    check(_lib.tq_sv_backward_pauli(ctx.h, _dt(states), ct.byref(spec.c), spec.gates.ctypes.data,
                                    spec.n_params.ctypes.data, params.data_ptr(), states.data_ptr(), pt.ctypes.data,
                                    int(pt.shape[0]), int(n_obs), grad_out.data_ptr(), grad.data_ptr(), ct.byref(o),
                                    work.data_ptr(), ct.c_int64(work.numel()), _stream()))
    return grad


def sv_backward_workspace(states, spec: BatchSpec, terms, n_obs, mode=0, tile_bits=0, reg_bits=0, ctx=None):
    """Workspace bytes tq_sv_backward needs for this batch (tq_sv_backward_workspace)."""
    ctx = ctx or context(states.device.index)
    terms = np.ascontiguousarray(terms, dtype=W.ZTERM_DTYPE)
    o = _opts(mode, tile_bits, reg_bits, 0)
    need = _lib.tq_sv_backward_workspace(ctx.h, _dt(states), ct.byref(spec.c), spec.gates.ctypes.data,
                                         spec.n_params.ctypes.data, terms.ctypes.data, int(terms.shape[0]),
                                         int(n_obs), ct.byref(o))
    if need < 0:
        raise TQError(1, last_error())
    return int(need)


def init_states(states, spec: BatchSpec, basis=0, ctx=None):
    """Write |basis> into every circuit's state (tq_sv_init)."""
    if not states.is_cuda or not states.is_contiguous() or states.numel() < spec.total_amps:
        raise ValueError("states must be a contiguous CUDA tensor covering the batch")
    ctx = ctx or context(states.device.index)
    check(_lib.tq_sv_init(ctx.h, _dt(states), ct.byref(spec.c), ct.c_int64(int(basis)), states.data_ptr(), _stream()))
    return states


def zero_states(spec: BatchSpec, dtype, device="cuda"):
    """New state tensor holding |0..0> for every circuit of the batch."""
    import torch
    st = torch.empty(spec.total_amps, dtype=dtype, device=device)
    return init_states(st, spec, 0)


# ---- compiled batches (tq_svb_*) ------------------------------------------------------------
class SvbOpts(ct.Structure):
    _fields_ = [(k, ct.c_int32) for k in ("tile_bits", "reg_bits", "coal_bits", "adj_tile_bits", "adj_reg_bits",
                                          "adj_coal_bits", "init", "graph")]


_lib.tq_svb_create.argtypes = [_vp, ct.c_int, ct.POINTER(Batch), _vp, _vp, _vp, _i32, _i32, ct.POINTER(SvbOpts),
                               ct.POINTER(_vp)]
_lib.tq_svb_create.restype = ct.c_int
_lib.tq_svb_destroy.argtypes = [_vp]
_lib.tq_svb_destroy.restype = None
_lib.tq_svb_forward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_svb_forward.restype = ct.c_int
_lib.tq_svb_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_svb_backward.restype = ct.c_int
_lib.tq_svb_autotune.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, _vp, ct.POINTER(SvbOpts), ct.POINTER(ct.c_double)]
_lib.tq_svb_autotune.restype = ct.c_int
_lib.tq_svb_info.argtypes = [_vp, ct.POINTER(ct.c_int64)]
_lib.tq_svb_info.restype = ct.c_int

SVB_INFO_FIELDS = ("levels", "items", "adj_levels", "adj_items", "graph_captures", "graph_replays", "tile_bits",
                   "reg_bits")


class SVBatch:
    """A batch of circuits compiled once (tq_svb_create) and run many times: forward
    (initial |0..0> unless ``init_from_states``, gate application, expectation values) and
    the adjoint backward, optionally replayed as HIP graphs (``graph=True``)."""

    def __init__(self, spec: BatchSpec, terms, n_obs, c128=False, graph=False, init_from_states=False,
                 tile_bits=0, reg_bits=0, adj_tile_bits=0, adj_reg_bits=0, ctx=None):
        self.spec = spec
        self.terms = np.ascontiguousarray(terms, dtype=W.ZTERM_DTYPE)
        self.n_obs = int(n_obs)
        self.c128 = bool(c128)
        self.ctx = ctx or context()
        o = SvbOpts(int(tile_bits), int(reg_bits), 0, int(adj_tile_bits), int(adj_reg_bits), 0,
                    1 if init_from_states else 0, 1 if graph else 0)
        h = _vp()
        check(_lib.tq_svb_create(self.ctx.h, TQ_C128 if c128 else TQ_C64, ct.byref(spec.c), spec.gates.ctypes.data,
                                 spec.n_params.ctypes.data, self.terms.ctypes.data, int(self.terms.shape[0]),
                                 self.n_obs, ct.byref(o), ct.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.tq_svb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dtypes(self):
        import torch
        return (torch.complex128, torch.float64) if self.c128 else (torch.complex64, torch.float32)

    def new_states(self, device="cuda"):
        import torch
        return torch.empty(self.spec.total_amps, dtype=self._dtypes()[0], device=device)

    def forward(self, params, states, out=None, with_expval=True):
        """Runs the batch; returns the [count, n_obs] expectation values (or None)."""
        import torch
        cdt, rdt = self._dtypes()
        if states.dtype != cdt:
            raise ValueError(f"states must be {cdt}")
        _check_tensors(states, params, self.spec)
        if with_expval and out is None:
            out = torch.empty((self.spec.count, self.n_obs), dtype=rdt, device=states.device)
        check(_lib.tq_svb_forward(self.ctx.h, self.h, params.data_ptr(), states.data_ptr(),
                                  out.data_ptr() if with_expval else None, _stream()))
        return out if with_expval else None

    def backward(self, params, states, grad_out, grad=None):
        """Adjoint gradients in the layout of params."""
        import torch
        _check_tensors(states, params, self.spec)
        if grad_out.dtype != params.dtype or not grad_out.is_contiguous() or \
                grad_out.numel() < self.spec.count * self.n_obs:
            raise ValueError(f"grad_out must be a contiguous {params.dtype} tensor of {self.spec.count} x {self.n_obs}")
        if grad is None:
            grad = torch.zeros_like(params)
        check(_lib.tq_svb_backward(self.ctx.h, self.h, params.data_ptr(), states.data_ptr(), grad_out.data_ptr(),
                                   grad.data_ptr(), _stream()))
        return grad

    def autotune(self, params, states, which=0, reps=3):
        """Times every candidate shape on the device and keeps the fastest; returns
        (tile_bits, reg_bits, ms)."""
        best = SvbOpts()
        ms = ct.c_double()
        check(_lib.tq_svb_autotune(self.ctx.h, self.h, params.data_ptr(), states.data_ptr(), int(which), int(reps),
                                   _stream(), ct.byref(best), ct.byref(ms)))
        if which == 0:
            return best.tile_bits, best.reg_bits, ms.value
        return best.adj_tile_bits, best.adj_reg_bits, ms.value

    @property
    def info(self):
        out = (ct.c_int64 * 8)()
        check(_lib.tq_svb_info(self.h, out))
        return dict(zip(SVB_INFO_FIELDS, [int(v) for v in out]))


# ---- tensor-network mode -------------------------------------------------------------------
class TnDesc(ct.Structure):
    _fields_ = [("n_leaves", ct.c_int32), ("leaf_rank", ct.c_void_p), ("leaf_inds", ct.c_void_p),
                ("pairs", ct.c_void_p), ("n_sliced", ct.c_int32), ("sliced", ct.c_void_p), ("n_out", ct.c_int32),
                ("out_inds", ct.c_void_p), ("dtype", ct.c_int32), ("slice_group", ct.c_int64),
                ("mem_budget", ct.c_int64), ("store_policy", ct.c_int32), ("_pad", ct.c_int32)]


TN_RECOMPUTE, TN_STORE, TN_AUTO = 0, 1, 2


TN_LEAF_DTYPE = np.dtype([("kind", "<i4"), ("gate", "<i4"), ("conj", "<i2"), ("flip", "<u2"), ("const_off", "<i4")])
assert TN_LEAF_DTYPE.itemsize == 16

_lib.tq_tn_plan_create.argtypes = [_vp, ct.POINTER(TnDesc), ct.POINTER(_vp)]
_lib.tq_tn_plan_create.restype = ct.c_int
_lib.tq_tn_plan_destroy.argtypes = [_vp]
_lib.tq_tn_plan_destroy.restype = None
_lib.tq_tn_leaf_elems.argtypes = [_vp]
_lib.tq_tn_leaf_elems.restype = ct.c_int64
_lib.tq_tn_leaf_offset.argtypes = [_vp, _i32]
_lib.tq_tn_leaf_offset.restype = ct.c_int64
_lib.tq_tn_plan_segments.argtypes = [_vp, ct.POINTER(ct.c_int64)]
_lib.tq_tn_plan_segments.restype = ct.c_int
_lib.tq_tn_plan_stores.argtypes = [_vp]
_lib.tq_tn_plan_stores.restype = ct.c_int32
_lib.tq_tn_workspace.argtypes = [_vp, _i32]
_lib.tq_tn_workspace.restype = ct.c_int64
_lib.tq_tn_plan_info.argtypes = [_vp, ct.POINTER(ct.c_int64)]
_lib.tq_tn_plan_info.restype = ct.c_int
_lib.tq_tn_contract.argtypes = [_vp, _vp, _vp, _vp, _vp, ct.c_int64, _vp]
_lib.tq_tn_contract.restype = ct.c_int
_lib.tq_tn_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ct.c_int64, _vp]
_lib.tq_tn_backward.restype = ct.c_int
_lib.tq_tn_build_leaves.argtypes = [_vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp]
_lib.tq_tn_build_leaves.restype = ct.c_int
_lib.tq_tn_param_grad.argtypes = [_vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp]
_lib.tq_tn_param_grad.restype = ct.c_int
_lib.tq_tn_build_leaves_batch.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_tn_build_leaves_batch.restype = ct.c_int
_lib.tq_tn_param_grad_batch.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_tn_param_grad_batch.restype = ct.c_int

TN_INFO_FIELDS = ("steps", "direct_steps", "gemm_steps", "slices", "slice_group", "flops", "gemm_flops",
                  "max_elems")


class TnPlan:
    """Owns a tq_tn_plan built from leaf index lists, an SSA tree and sliced indices."""

    def __init__(self, leaf_inds, pairs, sliced=(), out_inds=(), c128=False, slice_group=0, mem_budget=0,
                 ctx=None, store_policy=TN_RECOMPUTE, host_only=False):
        # host_only: planned without a context (no device needed); it can be queried, not run
        self.ctx = None if host_only else (ctx or context())
        self.c128 = bool(c128)
        ranks = np.array([len(x) for x in leaf_inds], dtype=np.int32)
        flat = np.array([i for x in leaf_inds for i in x] or [0], dtype=np.int32)
        pr = np.array([v for p in pairs for v in p] or [0], dtype=np.int32)
        sl = np.array(list(sliced) or [0], dtype=np.int32)
        oi = np.array(list(out_inds) or [0], dtype=np.int32)
        self._keep = (ranks, flat, pr, sl, oi)
        d = TnDesc(len(leaf_inds), ranks.ctypes.data, flat.ctypes.data, pr.ctypes.data, len(sliced), sl.ctypes.data,
                   len(out_inds), oi.ctypes.data, TQ_C128 if c128 else TQ_C64, int(slice_group), int(mem_budget),
                   int(store_policy), 0)
        h = _vp()
        check(_lib.tq_tn_plan_create(self.ctx.h if self.ctx else None, ct.byref(d), ct.byref(h)))
        self.h = h
        self.n_leaves = len(leaf_inds)
        self.leaf_elems = int(_lib.tq_tn_leaf_elems(h))
        self.leaf_offsets = [int(_lib.tq_tn_leaf_offset(h, i)) for i in range(self.n_leaves)]
        self.n_out = len(out_inds)
        out = (ct.c_int64 * 8)()
        check(_lib.tq_tn_plan_info(h, out))
        self.info = dict(zip(TN_INFO_FIELDS, [int(v) for v in out]))
        self.stores = bool(_lib.tq_tn_plan_stores(h))
        seg = (ct.c_int64 * 4)()
        check(_lib.tq_tn_plan_segments(h, seg))
        self.info.update(zip(("fwd_segments", "fwd_fused", "bwd_segments", "bwd_fused"), [int(v) for v in seg]))
        # a plan never changes: its workspace sizes are read once
        self._ws_bytes = (int(_lib.tq_tn_workspace(h, 0)), int(_lib.tq_tn_workspace(h, 1)))

    def workspace_bytes(self, backward=False):
        return self._ws_bytes[1 if backward else 0]

    @property
    def ctx_h(self):
        # a host-only plan is passed with the default context; the library refuses to run it
        return (self.ctx or context()).h

    def __del__(self):
        try:
            if self.h:
                _lib.tq_tn_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass


def _ws(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def tn_contract(plan: TnPlan, leaves, work=None):
    """Value of the network (2^n_out complex) from the packed leaf buffer (tq_tn_contract)."""
    import torch
    cdt = torch.complex128 if plan.c128 else torch.complex64
    if leaves.dtype != cdt or not leaves.is_cuda or leaves.numel() < plan.leaf_elems:
        raise ValueError("leaves must be a CUDA tensor of the plan's dtype covering the packed leaf buffer")
    leaves = leaves.contiguous()
    out = torch.empty(1 << plan.n_out, dtype=cdt, device=leaves.device)
    need = plan.workspace_bytes(False)
    work = work if work is not None and work.numel() >= need else _ws(need, leaves.device)
    check(_lib.tq_tn_contract(plan.ctx_h, plan.h, leaves.data_ptr(), out.data_ptr(), work.data_ptr(), need,
                              _stream()))
    return out


def tn_backward(plan: TnPlan, leaves, grad_out, work=None):
    """Leaf environments scaled by grad_out, packed like the leaves (tq_tn_backward)."""
    import torch
    cdt = torch.complex128 if plan.c128 else torch.complex64
    leaves = leaves.contiguous()
    g = grad_out.to(device=leaves.device, dtype=cdt).contiguous()
    if g.numel() < (1 << plan.n_out):
        raise ValueError("grad_out too small")
    grad = torch.empty(plan.leaf_elems, dtype=cdt, device=leaves.device)
    need = plan.workspace_bytes(True)
    work = work if work is not None and work.numel() >= need else _ws(need, leaves.device)
    check(_lib.tq_tn_backward(plan.ctx_h, plan.h, leaves.data_ptr(), g.data_ptr(), grad.data_ptr(), work.data_ptr(),
                              need, _stream()))
    return grad


_lib.tq_tn_contract_batch.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_tn_contract_batch.restype = ct.c_int
_lib.tq_tn_backward_batch.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tq_tn_backward_batch.restype = ct.c_int


def _ptrs(xs):
    return (ct.c_void_p * max(1, len(xs)))(*[ct.c_void_p(x) for x in xs])


def tn_contract_batch(plans, leaves, works=None):
    """Values of many networks (tq_tn_contract_batch); returns one output tensor per plan."""
    import torch
    outs, ws = [], []
    for k, (pl, lv) in enumerate(zip(plans, leaves)):
        cdt = torch.complex128 if pl.c128 else torch.complex64
        if lv.dtype != cdt or not lv.is_cuda or not lv.is_contiguous() or lv.numel() < pl.leaf_elems:
            raise ValueError(f"leaves of network {k} do not fit its plan")
        outs.append(torch.empty(1 << pl.n_out, dtype=cdt, device=lv.device))
        need = pl.workspace_bytes(False)
        ws.append(works[k] if works is not None and works[k].numel() >= need else _ws(need, lv.device))
    need = (ct.c_int64 * max(1, len(plans)))(*[pl.workspace_bytes(False) for pl in plans])
    check(_lib.tq_tn_contract_batch(plans[0].ctx_h if plans else context().h, len(plans),
                                    _ptrs([pl.h.value for pl in plans]), _ptrs([x.data_ptr() for x in leaves]),
                                    _ptrs([o.data_ptr() for o in outs]), _ptrs([w.data_ptr() for w in ws]), need,
                                    _stream()))
    return outs


def tn_backward_batch(plans, leaves, grad_outs, works=None):
    """Leaf environments of many networks (tq_tn_backward_batch), one packed tensor per plan."""
    import torch
    envs, ws, gs = [], [], []
    for k, (pl, lv, g) in enumerate(zip(plans, leaves, grad_outs)):
        cdt = torch.complex128 if pl.c128 else torch.complex64
        if lv.dtype != cdt or not lv.is_cuda or not lv.is_contiguous() or lv.numel() < pl.leaf_elems:
            raise ValueError(f"leaves of network {k} do not fit its plan")
        gs.append(g.to(device=lv.device, dtype=cdt).contiguous())
        envs.append(torch.empty(pl.leaf_elems, dtype=cdt, device=lv.device))
        need = pl.workspace_bytes(True)
        ws.append(works[k] if works is not None and works[k].numel() >= need else _ws(need, lv.device))
    need = (ct.c_int64 * max(1, len(plans)))(*[pl.workspace_bytes(True) for pl in plans])
    check(_lib.tq_tn_backward_batch(plans[0].ctx_h if plans else context().h, len(plans),
                                    _ptrs([pl.h.value for pl in plans]), _ptrs([x.data_ptr() for x in leaves]),
                                    _ptrs([g.data_ptr() for g in gs]), _ptrs([e.data_ptr() for e in envs]),
                                    _ptrs([w.data_ptr() for w in ws]), need, _stream()))
    return envs


def tn_build_leaves(plan: TnPlan, gates, leaf_specs, const_vals, params):
    """Packed leaf buffer of a circuit network from its parameters (tq_tn_build_leaves)."""
    import torch
    cdt = torch.complex128 if plan.c128 else torch.complex64
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    ls = np.ascontiguousarray(leaf_specs, dtype=TN_LEAF_DTYPE)
    cv = np.ascontiguousarray(np.asarray(const_vals, dtype=np.complex128).view(np.float64))
    out = torch.empty(plan.leaf_elems, dtype=cdt, device=params.device)
    check(_lib.tq_tn_build_leaves(plan.ctx_h, plan.h, g.ctypes.data, int(g.shape[0]), ls.ctypes.data,
                                  cv.ctypes.data, int(cv.shape[0] // 2), params.data_ptr(), out.data_ptr(),
                                  _stream()))
    return out


def tn_param_grad(plan: TnPlan, gates, leaf_specs, params, grad_leaves):
    """Re sum over leaves of env * dLeaf/dparam for every parameter (tq_tn_param_grad)."""
    import torch
    g = np.ascontiguousarray(gates, dtype=W.GATE_DTYPE)
    ls = np.ascontiguousarray(leaf_specs, dtype=TN_LEAF_DTYPE)
    out = torch.empty(params.numel(), dtype=params.dtype, device=params.device)
    check(_lib.tq_tn_param_grad(plan.ctx_h, plan.h, g.ctypes.data, int(g.shape[0]), ls.ctypes.data,
                                params.data_ptr(), int(params.numel()), grad_leaves.contiguous().data_ptr(),
                                out.data_ptr(), _stream()))
    return out


def _i32s(xs):
    return (ct.c_int32 * max(1, len(xs)))(*[int(x) for x in xs])


def tn_build_leaves_batch(plans, gates_list, specs_list, consts_list, params_list):
    """Packed leaf buffers of many networks in one launch (tq_tn_build_leaves_batch); every
    plan must have the same dtype. Returns one leaf tensor per plan."""
    import torch
    if not plans:
        return []
    cdt = torch.complex128 if plans[0].c128 else torch.complex64
    gs = [np.ascontiguousarray(g, dtype=W.GATE_DTYPE) for g in gates_list]
    ls = [np.ascontiguousarray(x, dtype=TN_LEAF_DTYPE) for x in specs_list]
    cv = [np.ascontiguousarray(np.asarray(c, dtype=np.complex128).view(np.float64)) for c in consts_list]
    outs = [torch.empty(pl.leaf_elems, dtype=cdt, device=q.device) for pl, q in zip(plans, params_list)]
    check(_lib.tq_tn_build_leaves_batch(plans[0].ctx_h, len(plans), _ptrs([pl.h.value for pl in plans]),
                                        _ptrs([g.ctypes.data for g in gs]), _i32s([g.shape[0] for g in gs]),
                                        _ptrs([x.ctypes.data for x in ls]), _ptrs([c.ctypes.data for c in cv]),
                                        _i32s([c.shape[0] // 2 for c in cv]),
                                        _ptrs([q.data_ptr() for q in params_list]),
                                        _ptrs([o.data_ptr() for o in outs]), _stream()))
    return outs


def tn_param_grad_batch(plans, gates_list, specs_list, params_list, grad_leaves_list):
    """Parameter gradients of many networks in one launch (tq_tn_param_grad_batch)."""
    import torch
    if not plans:
        return []
    gs = [np.ascontiguousarray(g, dtype=W.GATE_DTYPE) for g in gates_list]
    ls = [np.ascontiguousarray(x, dtype=TN_LEAF_DTYPE) for x in specs_list]
    env = [e.contiguous() for e in grad_leaves_list]
    outs = [torch.empty(q.numel(), dtype=q.dtype, device=q.device) for q in params_list]
    check(_lib.tq_tn_param_grad_batch(plans[0].ctx_h, len(plans), _ptrs([pl.h.value for pl in plans]),
                                      _ptrs([g.ctypes.data for g in gs]), _i32s([g.shape[0] for g in gs]),
                                      _ptrs([x.ctypes.data for x in ls]), _ptrs([q.data_ptr() for q in params_list]),
                                      _i32s([q.numel() for q in params_list]), _ptrs([e.data_ptr() for e in env]),
                                      _ptrs([o.data_ptr() for o in outs]), _stream()))
    return outs


# ---- cost-model MLP (tq_mlp_*) ---------------------------------------------------------------
class MlpDesc(ct.Structure):
    _fields_ = [("n_layers", ct.c_int32), ("sizes", ct.c_int32 * 9)]


_lib.tq_mlp_param_count.argtypes = [ct.POINTER(MlpDesc)]
_lib.tq_mlp_param_count.restype = ct.c_int64
_lib.tq_mlp_workspace.argtypes = [ct.POINTER(MlpDesc), _i32]
_lib.tq_mlp_workspace.restype = ct.c_int64
_lib.tq_mlp_forward.argtypes = [_vp, ct.POINTER(MlpDesc), _vp, _vp, _i32, _vp, _vp, ct.c_int64, _vp]
_lib.tq_mlp_forward.restype = ct.c_int
_lib.tq_mlp_train_step.argtypes = [_vp, ct.POINTER(MlpDesc), _vp, _vp, _vp, _i32, ct.c_float, ct.c_float, ct.c_float,
                                   ct.c_float, _vp, _vp, _i32, _vp, _vp, _vp, ct.c_int64, _vp]
_lib.tq_mlp_train_step.restype = ct.c_int


def mlp_desc(sizes):
    d = MlpDesc()
    d.n_layers = len(sizes) - 1
    for i, v in enumerate(sizes):
        d.sizes[i] = int(v)
    return d


def mlp_param_count(sizes):
    n = int(_lib.tq_mlp_param_count(ct.byref(mlp_desc(sizes))))
    if n < 0:
        raise TQError(1, last_error())
    return n


def _f32(t, name):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA float32 tensor")


def mlp_forward(sizes, params, x, ctx=None):
    """[batch] outputs of the MLP on x [batch, sizes[0]] (tq_mlp_forward)."""
    import torch
    _f32(params, "params")
    _f32(x, "x")
    d = mlp_desc(sizes)
    B = int(x.shape[0])
    if x.numel() != B * sizes[0] or params.numel() != mlp_param_count(sizes):
        raise ValueError("shape mismatch")
    ctx = ctx or context(x.device.index)
    y = torch.empty(B, dtype=torch.float32, device=x.device)
    need = int(_lib.tq_mlp_workspace(ct.byref(d), B))
    ws = _ws(need, x.device)
    check(_lib.tq_mlp_forward(ctx.h, ct.byref(d), params.data_ptr(), x.data_ptr(), B, y.data_ptr(), ws.data_ptr(),
                              need, _stream()))
    return y


def mlp_train_step(sizes, params, m, v, t, x, y, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_grad=False,
                   ctx=None):
    """One Adam step on the MSE of the MLP (tq_mlp_train_step); returns (loss tensor [1], grad or None)."""
    import torch
    for a, nm in ((params, "params"), (m, "m"), (v, "v"), (x, "x"), (y, "y")):
        _f32(a, nm)
    d = mlp_desc(sizes)
    B = int(x.shape[0])
    P = mlp_param_count(sizes)
    if params.numel() != P or m.numel() != P or v.numel() != P or y.numel() != B or x.numel() != B * sizes[0]:
        raise ValueError("shape mismatch")
    ctx = ctx or context(x.device.index)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(P, dtype=torch.float32, device=x.device) if want_grad else None
    need = int(_lib.tq_mlp_workspace(ct.byref(d), B))
    ws = _ws(need, x.device)
    check(_lib.tq_mlp_train_step(ctx.h, ct.byref(d), params.data_ptr(), m.data_ptr(), v.data_ptr(), int(t),
                                 float(lr), float(beta1), float(beta2), float(eps), x.data_ptr(), y.data_ptr(), B,
                                 loss.data_ptr(), grad.data_ptr() if want_grad else None, ws.data_ptr(), need,
                                 _stream()))
    return loss, grad
