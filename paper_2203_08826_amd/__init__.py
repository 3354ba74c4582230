"""MI355X state-vector simulator: Python binding of libqsv.so.

Every function here has the name of the C entry point it calls
(include/qsv.h) and only marshals arguments: torch tensors supply device
memory and the current HIP stream; gate descriptions become ``qsv_gate``
structs.  All simulation work runs in the library's HIP kernels; there is no
CPU fallback -- without the built library every call raises.

Gate descriptions are dicts ``{"name", "targets", "controls", "params"}``
(plus ``"matrix"`` for UNITARY and ``"diag"`` for DIAG), qubit q = bit q of
the amplitude index, targets[0] = most significant bit of a gate matrix.
"""
import ctypes

import numpy as np

from . import _abi
from ._abi import (COST_FEATURES, GATE_KINDS, PLAN_GREEDY, PLAN_LEARNED, PLAN_PASSES, PLAN_PER_GATE,
                   QSV_C64, QSV_C128, QsvError, QsvGate, QsvPlanOptions, QsvPlanStats, check, load)

__all__ = [name for name in _abi.SIGNATURES] + [
    "load", "QsvError", "Plan", "gates_to_c", "QSV_C64", "QSV_C128", "PLAN_PER_GATE", "PLAN_GREEDY",
    "PLAN_PASSES", "PLAN_LEARNED"]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex64:
        return QSV_C64
    if t.dtype == torch.complex128:
        return QSV_C128
    raise TypeError("state must be complex64 or complex128, got %s" % t.dtype)


def _state(t):
    if not t.is_cuda:
        raise ValueError("state must be a device tensor (no CPU fallback)")
    if not t.is_contiguous():
        raise ValueError("state must be contiguous")
    size = t.numel()
    n = size.bit_length() - 1
    if size < 2 or size != 1 << n:
        raise ValueError("state length must be a power of two >= 2")
    return ctypes.c_void_p(t.data_ptr()), n, _dtype_code(t)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ints(xs):
    xs = [int(x) for x in xs]
    arr = (ctypes.c_int * max(1, len(xs)))(*xs)
    return arr, len(xs)


def _host_complex(m, dtype_code):
    np_dt = np.complex64 if dtype_code == QSV_C64 else np.complex128
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128).astype(np_dt))


def _dev_out(shape, out, dtype=None):
    torch = _torch()
    dtype = dtype or torch.float64
    if out is None:
        out = torch.empty(shape, dtype=dtype, device="cuda")
    if not out.is_cuda or out.dtype != dtype or not out.is_contiguous() or out.numel() < int(np.prod(shape)):
        raise ValueError("out must be a contiguous device tensor of %s with %s elements" % (dtype, shape))
    return out


# ------------------------------------------------------------------ misc

def qsv_abi_version():
    return load().qsv_abi_version()


def qsv_status_string(status):
    return load().qsv_status_string(int(status)).decode()


def qsv_last_error():
    return load().qsv_last_error().decode(errors="replace")


def qsv_memory_stats(reset_peak=False):
    """(current, peak) bytes of device memory the library holds for itself."""
    cur, peak = ctypes.c_uint64(), ctypes.c_uint64()
    check("qsv_memory_stats", load().qsv_memory_stats(ctypes.byref(cur), ctypes.byref(peak), int(bool(reset_peak))))
    return cur.value, peak.value


def qsv_validate(n, dtype, targets, controls=()):
    """Host-only validation; returns the status code (no exception)."""
    t, k = _ints(targets)
    c, nc = _ints(controls)
    return load().qsv_validate(int(n), int(dtype), t, k, c, nc)


def qsv_group_index_host(n, bits, first, count):
    b, m = _ints(bits)
    out = np.empty(int(count), dtype=np.uint64)
    check("qsv_group_index_host",
          load().qsv_group_index_host(int(n), b, m, int(first), int(count), out.ctypes.data))
    return out


# ------------------------------------------------------------------ gates

def qsv_apply_matrix(state, gate, targets, controls=(), stream=None):
    p, n, dt = _state(state)
    g = _host_complex(gate, dt)
    t, k = _ints(targets)
    c, nc = _ints(controls)
    if g.shape != (1 << k, 1 << k):
        raise ValueError("gate must be %dx%d" % (1 << k, 1 << k))
    check("qsv_apply_matrix", load().qsv_apply_matrix(p, n, dt, g.ctypes.data, t, k, c, nc, _stream(stream)))


def qsv_apply_x(state, target, controls=(), stream=None):
    p, n, dt = _state(state)
    c, nc = _ints(controls)
    check("qsv_apply_x", load().qsv_apply_x(p, n, dt, int(target), c, nc, _stream(stream)))


def qsv_apply_y(state, target, controls=(), stream=None):
    p, n, dt = _state(state)
    c, nc = _ints(controls)
    check("qsv_apply_y", load().qsv_apply_y(p, n, dt, int(target), c, nc, _stream(stream)))


def qsv_apply_z(state, target, controls=(), stream=None):
    p, n, dt = _state(state)
    c, nc = _ints(controls)
    check("qsv_apply_z", load().qsv_apply_z(p, n, dt, int(target), c, nc, _stream(stream)))


def qsv_apply_swap(state, t0, t1, controls=(), stream=None):
    p, n, dt = _state(state)
    c, nc = _ints(controls)
    check("qsv_apply_swap", load().qsv_apply_swap(p, n, dt, int(t0), int(t1), c, nc, _stream(stream)))


def qsv_apply_phase(state, target, phi, controls=(), stream=None):
    p, n, dt = _state(state)
    c, nc = _ints(controls)
    check("qsv_apply_phase", load().qsv_apply_phase(p, n, dt, int(target), float(phi), c, nc, _stream(stream)))


def qsv_apply_diagonal(state, diag, targets, controls=(), stream=None):
    p, n, dt = _state(state)
    d = _host_complex(diag, dt).reshape(-1)
    t, k = _ints(targets)
    c, nc = _ints(controls)
    if d.size != 1 << k:
        raise ValueError("diag must have 2^k entries")
    check("qsv_apply_diagonal", load().qsv_apply_diagonal(p, n, dt, d.ctypes.data, t, k, c, nc, _stream(stream)))


def qsv_apply_fsim(state, t0, t1, theta, phi, stream=None):
    p, n, dt = _state(state)
    check("qsv_apply_fsim", load().qsv_apply_fsim(p, n, dt, int(t0), int(t1), float(theta), float(phi),
                                                  _stream(stream)))


# ------------------------------------------------------------------ circuits

def qsv_scale(state, factor, stream=None):
    """state <- factor * state (complex factor), in place."""
    p, n, dt = _state(state)
    f = complex(factor)
    check("qsv_scale", load().qsv_scale(p, n, dt, f.real, f.imag, _stream(stream)))


def gates_to_c(circuit):
    """Array of qsv_gate for a list of gate dicts, plus the host buffers it points to."""
    arr = (QsvGate * max(1, len(circuit)))()
    keep = []
    for i, g in enumerate(circuit):
        name = g["name"]
        if name not in GATE_KINDS:
            raise ValueError("unknown gate name %r" % name)
        s = arr[i]
        s.kind = GATE_KINDS[name]
        tg = list(g["targets"])
        cs = list(g.get("controls", []))
        if len(tg) > _abi.MAX_TARGETS or len(cs) > _abi.MAX_CONTROLS:
            raise ValueError("gate has too many targets or controls")
        s.k, s.c = len(tg), len(cs)
        for j, q in enumerate(tg):
            s.targets[j] = int(q)
        for j, q in enumerate(cs):
            s.controls[j] = int(q)
        ps = list(g.get("params", []))
        for j in range(min(2, len(ps))):
            s.params[j] = float(ps[j])
        if s.kind == 0:
            m = np.ascontiguousarray(np.asarray(g["matrix"], dtype=np.complex128))
            keep.append(m)
            s.data = m.ctypes.data
        elif s.kind == GATE_KINDS["DIAG"]:
            d = np.ascontiguousarray(np.asarray(g["diag"], dtype=np.complex128).reshape(-1))
            keep.append(d)
            s.data = d.ctypes.data
    return arr, keep


def qsv_gate_matrix(gate):
    """Host-only: complex128 target block of a gate dict as built by the library."""
    arr, keep = gates_to_c([gate])
    k = arr[0].k
    out = np.empty((1 << k, 1 << k), dtype=np.complex128)
    check("qsv_gate_matrix", load().qsv_gate_matrix(ctypes.byref(arr[0]), out.ctypes.data))
    del keep
    return out


class Plan:
    """Owner of a ``qsv_plan*`` (qsv_plan_create / _execute / _stats_get / _destroy)."""

    def __init__(self, handle, ngates):
        self._h = handle
        self.ngates = ngates

    def stats(self):
        return qsv_plan_stats_get(self)

    def __del__(self):
        try:
            if self._h:
                load().qsv_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def qsv_plan_create(n, dtype, circuit, mode=PLAN_PER_GATE, kmax=2, local_bits=0, use_mfma=1, jit=0):
    arr, keep = gates_to_c(circuit)
    opts = QsvPlanOptions(int(mode), int(kmax), int(local_bits), int(use_mfma), int(jit))
    h = ctypes.c_void_p()
    check("qsv_plan_create", load().qsv_plan_create(int(n), int(dtype), arr, len(circuit), ctypes.byref(opts),
                                                    ctypes.byref(h)))
    del keep
    return Plan(h, len(circuit))


def qsv_plan_stats_get(plan):
    s = QsvPlanStats()
    check("qsv_plan_stats_get", load().qsv_plan_stats_get(plan._h, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in QsvPlanStats._fields_}


def qsv_plan_blocks(plan):
    out = (ctypes.c_int * max(1, plan.ngates))()
    check("qsv_plan_blocks", load().qsv_plan_blocks(plan._h, out, plan.ngates))
    return list(out)[:plan.ngates]


def qsv_plan_execute(plan, state, stream=None):
    p, n, dt = _state(state)
    check("qsv_plan_execute", load().qsv_plan_execute(plan._h, p, _stream(stream)))


def qsv_plan_execute_ops(plan, state, first, count, stream=None):
    p, n, dt = _state(state)
    check("qsv_plan_execute_ops", load().qsv_plan_execute_ops(plan._h, p, int(first), int(count), _stream(stream)))


def qsv_plan_op_info(plan, index):
    kind = ctypes.c_int()
    b = ctypes.c_double()
    f = ctypes.c_double()
    check("qsv_plan_op_info", load().qsv_plan_op_info(plan._h, int(index), ctypes.byref(kind), ctypes.byref(b),
                                                      ctypes.byref(f)))
    return {"kind": kind.value, "bytes": b.value, "flops": f.value}


def qsv_plan_op_program(plan, index):
    """Host-only: serialised LDS-pass program of op `index` as bytes."""
    size = ctypes.c_size_t()
    check("qsv_plan_op_program", load().qsv_plan_op_program(plan._h, int(index), None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(size.value)
    check("qsv_plan_op_program", load().qsv_plan_op_program(plan._h, int(index), buf, size.value, ctypes.byref(size)))
    return buf.raw[:size.value]


def qsv_plan_op_source(plan, index):
    """HIP source of the compiled kernel of LDS-pass op `index` (host only)."""
    size = ctypes.c_size_t(0)
    check("qsv_plan_op_source", load().qsv_plan_op_source(plan._h, int(index), None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(size.value)
    check("qsv_plan_op_source", load().qsv_plan_op_source(plan._h, int(index), buf, size.value, ctypes.byref(size)))
    return buf.value.decode()


def qsv_plan_op_gates(plan, index):
    """Circuit indices of the gates op `index` applies, in application order."""
    count = ctypes.c_size_t(0)
    check("qsv_plan_op_gates", load().qsv_plan_op_gates(plan._h, int(index), None, 0, ctypes.byref(count)))
    ids = (ctypes.c_int * max(count.value, 1))()
    check("qsv_plan_op_gates", load().qsv_plan_op_gates(plan._h, int(index), ids, count.value, ctypes.byref(count)))
    return [int(ids[i]) for i in range(count.value)]


def qsv_plan_destroy(plan):
    if plan._h:
        load().qsv_plan_destroy(plan._h)
        plan._h = None


def qsv_apply_block(state, gate, targets, stream=None):
    p, n, dt = _state(state)
    g = _host_complex(gate, dt)
    t, k = _ints(targets)
    check("qsv_apply_block", load().qsv_apply_block(p, n, dt, g.ctypes.data, t, k, _stream(stream)))


def qsv_run_pass(state, circuit, local_qubits, stream=None):
    p, n, dt = _state(state)
    arr, keep = gates_to_c(circuit)
    lq, nl = _ints(local_qubits)
    check("qsv_run_pass", load().qsv_run_pass(p, n, dt, arr, len(circuit), lq, nl, _stream(stream)))
    del keep


# ------------------------------------------------------------------ reductions

def qsv_probabilities(state, qubits, out=None, stream=None):
    p, n, dt = _state(state)
    q, r = _ints(qubits)
    out = _dev_out((1 << r,), out)
    check("qsv_probabilities", load().qsv_probabilities(p, n, dt, q, r, ctypes.c_void_p(out.data_ptr()),
                                                        _stream(stream)))
    return out


def qsv_probabilities_noalloc(state, qubits, out, stream=None):
    """qsv_probabilities without any allocation inside the library; `out`
    (float64 device tensor of 2^r entries) must be supplied."""
    torch = _torch()
    p, n, dt = _state(state)
    q, r = _ints(qubits)
    if out is None:
        raise ValueError("out must be supplied (this call allocates nothing)")
    out = _dev_out((1 << r,), out)
    check("qsv_probabilities_noalloc", load().qsv_probabilities_noalloc(
        p, n, dt, q, r, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qsv_norm2(state, out=None, stream=None):
    p, n, dt = _state(state)
    out = _dev_out((1,), out)
    check("qsv_norm2", load().qsv_norm2(p, n, dt, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qsv_inner(a, b, out=None, stream=None):
    pa, n, dt = _state(a)
    pb, nb, dtb = _state(b)
    if (nb, dtb) != (n, dt):
        raise ValueError("a and b must have the same size and dtype")
    out = _dev_out((2,), out)
    check("qsv_inner", load().qsv_inner(pa, pb, n, dt, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qsv_expval_zz_x(state, J=1.0, h=0.5, periodic=False, out=None, stream=None):
    p, n, dt = _state(state)
    out = _dev_out((1,), out)
    check("qsv_expval_zz_x", load().qsv_expval_zz_x(p, n, dt, float(J), float(h), int(bool(periodic)),
                                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qsv_apply_tfim(state, out, J=1.0, h=0.5, periodic=False, stream=None):
    p, n, dt = _state(state)
    po, no, dto = _state(out)
    if (no, dto) != (n, dt):
        raise ValueError("out must match state")
    check("qsv_apply_tfim", load().qsv_apply_tfim(p, po, n, dt, float(J), float(h), int(bool(periodic)),
                                                  _stream(stream)))
    return out


# ------------------------------------------------------------------ host-resident states

def qsv_sliced_run(host_state, circuit, local_qubits, active_qubits=2, mode=PLAN_PASSES, stream=None):
    """Run `circuit` on a state in host memory (a contiguous CPU tensor,
    complex64 or complex128, pinned for overlapped copies), slices of
    2^local_qubits amplitudes visiting the device; returns when the host
    state holds the result."""
    torch = _torch()
    t = host_state
    if t.is_cuda or not t.is_contiguous():
        raise ValueError("host_state must be a contiguous host tensor")
    size = t.numel()
    n = size.bit_length() - 1
    if size < 2 or size != 1 << n:
        raise ValueError("state length must be a power of two >= 2")
    dt = _dtype_code(t)
    arr, keep = gates_to_c(circuit)
    check("qsv_sliced_run", load().qsv_sliced_run(ctypes.c_void_p(t.data_ptr()), n, dt, arr, len(circuit),
                                                  int(local_qubits), int(active_qubits), int(mode), _stream(stream)))
    del keep
    return t


# ------------------------------------------------------------------ measurement

def _dptr(t, dtype, count, what):
    torch = _torch()
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < count:
        raise ValueError("%s must be a contiguous device tensor of %s with >= %d elements" % (what, dtype, count))
    return ctypes.c_void_p(t.data_ptr())


def qsv_collapse(state, qubits, outcome, prob_out=None, stream=None):
    """Collapse `state` in place onto `outcome` of `qubits`; returns a device
    float64 tensor holding the outcome's probability before re-normalisation."""
    torch = _torch()
    p, n, dt = _state(state)
    q, r = _ints(qubits)
    prob_out = _dev_out((1,), prob_out)
    check("qsv_collapse", load().qsv_collapse(p, n, dt, q, r, int(outcome), ctypes.c_void_p(prob_out.data_ptr()),
                                              _stream(stream)))
    return prob_out


def qsv_sample_cdf(probs, uniforms, cdf=None, samples=True, counts=True, stream=None):
    """Inverse-CDF samples of `probs` (device float64, 2^r) for device float64
    `uniforms`; returns (cdf, samples or None, counts or None)."""
    torch = _torch()
    R = probs.numel()
    r = R.bit_length() - 1
    if R < 2 or R != 1 << r:
        raise ValueError("probs must hold 2^r entries, r >= 1")
    ns = uniforms.numel()
    cdf = cdf if cdf is not None else torch.empty(R, dtype=torch.float64, device=probs.device)
    sm = torch.empty(ns, dtype=torch.int64, device=probs.device) if samples else None
    ct = torch.empty(R, dtype=torch.uint64, device=probs.device) if counts else None
    check("qsv_sample_cdf", load().qsv_sample_cdf(
        _dptr(probs, torch.float64, R, "probs"), r, _dptr(uniforms, torch.float64, ns, "uniforms"), ns,
        _dptr(cdf, torch.float64, R, "cdf"), _dptr(sm, torch.int64, ns, "samples"),
        _dptr(ct, torch.uint64, R, "counts"), _stream(stream)))
    return cdf, sm, ct


def qsv_sample_metropolis(probs, starts, proposals, uniforms, stream=None):
    """Metropolis frequencies: `starts` [C] int64, `proposals` [steps, C]
    int64, `uniforms` [steps, C] float64 (device); returns counts [2^r] uint64."""
    torch = _torch()
    R = probs.numel()
    r = R.bit_length() - 1
    if R < 2 or R != 1 << r:
        raise ValueError("probs must hold 2^r entries, r >= 1")
    C = starts.numel()
    steps = proposals.shape[0] if proposals.dim() == 2 else 0
    if proposals.numel() != steps * C or uniforms.numel() != steps * C:
        raise ValueError("proposals and uniforms must be [steps, chains]")
    counts = torch.empty(R, dtype=torch.uint64, device=probs.device)
    check("qsv_sample_metropolis", load().qsv_sample_metropolis(
        _dptr(probs, torch.float64, R, "probs"), r, _dptr(starts, torch.int64, C, "starts"),
        _dptr(proposals, torch.int64, steps * C, "proposals"), _dptr(uniforms, torch.float64, steps * C, "uniforms"),
        C, steps, _dptr(counts, torch.uint64, R, "counts"), _stream(stream)))
    return counts


# ------------------------------------------------------------------ density matrices

def _dm(rho):
    """(pointer, n, dtype) of a density matrix tensor of 2^(2n) entries."""
    p, n2, dt = _state(rho)
    if n2 % 2:
        raise ValueError("a density matrix holds 2^(2n) entries")
    return p, n2 // 2, dt


def qsv_dm_plan_create(n, dtype, circuit, mode=PLAN_PER_GATE, kmax=2, local_bits=0, use_mfma=1, jit=0):
    """Plan applying `circuit` to an n-qubit density matrix (rho -> G rho G^dag);
    run it with qsv_plan_execute on the 2^(2n)-entry rho."""
    arr, keep = gates_to_c(circuit)
    opts = QsvPlanOptions(int(mode), int(kmax), int(local_bits), int(use_mfma), int(jit))
    h = ctypes.c_void_p()
    check("qsv_dm_plan_create", load().qsv_dm_plan_create(int(n), int(dtype), arr, len(circuit), ctypes.byref(opts),
                                                          ctypes.byref(h)))
    del keep
    return Plan(h, 2 * len(circuit))


def qsv_dm_apply_channel(rho, kraus, target, stream=None):
    p, n, dt = _dm(rho)
    k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128).reshape(-1, 2, 2))
    check("qsv_dm_apply_channel", load().qsv_dm_apply_channel(p, n, dt, k.ctypes.data, k.shape[0], int(target),
                                                              _stream(stream)))


def qsv_dm_trace(rho, out=None, stream=None):
    p, n, dt = _dm(rho)
    out = _dev_out((2,), out)
    check("qsv_dm_trace", load().qsv_dm_trace(p, n, dt, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qsv_dm_probabilities(rho, qubits, out=None, stream=None):
    p, n, dt = _dm(rho)
    q, r = _ints(qubits)
    out = _dev_out((1 << r,), out)
    check("qsv_dm_probabilities", load().qsv_dm_probabilities(p, n, dt, q, r, ctypes.c_void_p(out.data_ptr()),
                                                              _stream(stream)))
    return out


# ------------------------------------------------------------------ adjoint

def qsv_adjoint_grad(psi, lam, circuit, out=None, stream=None):
    p, n, dt = _state(psi)
    pl, nl, dtl = _state(lam)
    if (nl, dtl) != (n, dt):
        raise ValueError("lam must match psi")
    arr, keep = gates_to_c(circuit)
    nparams = sum(1 for g in circuit if g["name"] in ("RX", "RY", "RZ"))
    out = _dev_out((max(1, nparams),), out)
    check("qsv_adjoint_grad", load().qsv_adjoint_grad(p, pl, n, dt, arr, len(circuit),
                                                      ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    del keep
    return out[:nparams]


# ------------------------------------------------------------------ MLP

def _fptr(t):
    torch = _torch()
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("MLP buffers must be contiguous float32 device tensors")
    return ctypes.c_void_p(t.data_ptr())


def qsv_mlp_param_count(sizes):
    s, m = _ints(sizes)
    return load().qsv_mlp_param_count(s, m - 1)


def qsv_mlp_forward(params, sizes, X, acts, pred, stream=None):
    s, m = _ints(sizes)
    check("qsv_mlp_forward", load().qsv_mlp_forward(_fptr(params), s, m - 1, _fptr(X), int(X.shape[0]),
                                                    _fptr(acts), _fptr(pred), _stream(stream)))


def qsv_mlp_backward(params, sizes, X, acts, pred, target, grads, scratch, stream=None):
    s, m = _ints(sizes)
    check("qsv_mlp_backward", load().qsv_mlp_backward(_fptr(params), s, m - 1, _fptr(X), int(X.shape[0]),
                                                      _fptr(acts), _fptr(pred), _fptr(target), _fptr(grads),
                                                      _fptr(scratch), _stream(stream)))


def qsv_mlp_adam(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check("qsv_mlp_adam", load().qsv_mlp_adam(_fptr(params), _fptr(grads), _fptr(m), _fptr(v), params.numel(),
                                              int(t), float(lr), float(beta1), float(beta2), float(eps),
                                              _stream(stream)))


def qsv_cost_model_set(params_host, sizes, feat_mean, feat_scale):
    s, m = _ints(sizes)
    p = np.ascontiguousarray(np.asarray(params_host, dtype=np.float32))
    mu = np.ascontiguousarray(np.asarray(feat_mean, dtype=np.float32))
    sc = np.ascontiguousarray(np.asarray(feat_scale, dtype=np.float32))
    check("qsv_cost_model_set", load().qsv_cost_model_set(p.ctypes.data, s, m - 1, mu.ctypes.data, sc.ctypes.data))


def qsv_cost_model_clear():
    s, _ = _ints([1])
    check("qsv_cost_model_set", load().qsv_cost_model_set(None, s, 0, None, None))


def qsv_plan_op_features(plan, index):
    """Host-only: raw cost-model features of op `index` of a plan."""
    out = np.empty(COST_FEATURES, dtype=np.float32)
    check("qsv_plan_op_features", load().qsv_plan_op_features(plan._h, int(index), out.ctypes.data))
    return out
