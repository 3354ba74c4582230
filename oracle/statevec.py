"""Oracle state-vector operations (complex128).  Test infrastructure only.

Gate application calls ``sim.c`` (Eq. 1 of the paper's introduction, out of
place).  Reductions use numpy's pairwise summation in float64.  The Kronecker
checker builds the full 2^n x 2^n operator of a gate for n <= 10.
"""
import ctypes
import os

import numpy as np

from . import build as _build
from . import gates as _gates

_lib = None


def lib():
    """Load ``_build/liboracle.so``, compiling it first if it is missing or stale."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        cp = ctypes.c_void_p
        L.oracle_apply_gate.argtypes = [ctypes.c_int, cp, cp, cp, cp, ctypes.c_int, cp, ctypes.c_int]
        L.oracle_apply_gate.restype = None
        L.oracle_abs2.argtypes = [ctypes.c_int, cp, cp]
        L.oracle_abs2.restype = None
        L.oracle_basis_state.argtypes = [ctypes.c_int, cp, ctypes.c_int64]
        L.oracle_basis_state.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads():
    return lib().oracle_num_threads()


def _ints(xs):
    a = np.ascontiguousarray(np.asarray(list(xs), dtype=np.int32))
    if a.size == 0:
        a = np.zeros(1, dtype=np.int32)
    return a


def apply_matrix(state, G, targets, controls=(), out=None):
    """Eq. 1 for one gate: return G applied to ``state`` (new array or ``out``).

    ``state`` is a complex128 vector of length 2^n; ``G`` the 2^k x 2^k target
    block (targets[0] = most significant bit of its index); the gate acts only
    where every control bit is 1.
    """
    state = np.ascontiguousarray(state, dtype=np.complex128)
    n = int(state.size).bit_length() - 1
    assert state.size == 1 << n
    G = np.ascontiguousarray(G, dtype=np.complex128)
    k = len(targets)
    assert G.shape == (1 << k, 1 << k)
    qs = list(targets) + list(controls)
    assert len(set(qs)) == len(qs) and all(0 <= q < n for q in qs)
    if out is None:
        out = np.empty_like(state)
    t = _ints(targets)
    c = _ints(controls)
    lib().oracle_apply_gate(n, state.ctypes.data, out.ctypes.data, G.ctypes.data,
                            t.ctypes.data, k, c.ctypes.data, len(controls))
    return out


def apply_gate(state, gate, out=None):
    """Apply a gate dict (see ``gates.target_matrix``) to ``state``."""
    return apply_matrix(state, _gates.target_matrix(gate), gate["targets"],
                        gate.get("controls", ()), out=out)


def run_circuit(state, circuit, copy=True):
    """Apply every gate of ``circuit`` in order; returns the final state.

    Two buffers are ping-ponged (out-of-place application, as Eq. 1 reads).
    """
    a = np.array(state, dtype=np.complex128, copy=True) if copy else state
    b = np.empty_like(a)
    for g in circuit:
        apply_gate(a, g, out=b)
        a, b = b, a
    return a


def basis_state(n, x):
    out = np.empty(1 << n, dtype=np.complex128)
    lib().oracle_basis_state(n, out.ctypes.data, int(x))
    return out


def abs2(state):
    state = np.ascontiguousarray(state, dtype=np.complex128)
    n = int(state.size).bit_length() - 1
    out = np.empty(state.size, dtype=np.float64)
    lib().oracle_abs2(n, state.ctypes.data, out.ctypes.data)
    return out


def norm2(state):
    """<psi|psi> in float64 (pairwise summation)."""
    return float(np.sum(abs2(state)))


def inner(a, b):
    """<a|b> = sum_i conj(a_i) b_i in complex128."""
    return complex(np.vdot(np.asarray(a, dtype=np.complex128), np.asarray(b, dtype=np.complex128)))


def infidelity(ref, psi):
    """1 - |<ref|psi>|^2 / (<ref|ref> <psi|psi>)."""
    ref = np.asarray(ref, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    ov = abs(np.vdot(ref, psi)) ** 2
    return float(1.0 - ov / (np.vdot(ref, ref).real * np.vdot(psi, psi).real))


def probabilities(state, qubits):
    """Measurement probabilities of ``qubits`` (methodology section: measurement).

    p(m) = sum over all amplitudes whose measured bits spell m of |psi_i|^2,
    with m = sum_j b_{qubits[j]} 2^{r-1-j} (qubits[0] is the most significant
    bit of the outcome index).  Float64 result of length 2^r.
    """
    p = abs2(state)
    n = int(p.size).bit_length() - 1
    qubits = list(qubits)
    # numpy axis a of the (2,)*n view is bit n-1-a of the index
    t = p.reshape((2,) * n)
    keep_axes = [n - 1 - q for q in qubits]
    other = tuple(a for a in range(n) if a not in keep_axes)
    s = t.sum(axis=other) if other else t
    # remaining axes appear in increasing axis order; move them into
    # qubits order (qubits[0] first = most significant)
    remaining = sorted(keep_axes)
    order = [remaining.index(a) for a in keep_axes]
    return np.ascontiguousarray(np.transpose(s, order)).reshape(-1)


def zz_diag(n, periodic=False):
    """Diagonal of sum_i Z_i Z_{i+1} (open chain unless ``periodic``)."""
    idx = np.arange(1 << n, dtype=np.int64)
    d = np.zeros(1 << n, dtype=np.float64)
    pairs = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        pairs.append((n - 1, 0))
    for a, b in pairs:
        par = ((idx >> a) ^ (idx >> b)) & 1
        d += 1.0 - 2.0 * par
    return d


def apply_h_tfim(state, J=1.0, h=0.5, periodic=False):
    """H psi for H = J sum Z_i Z_{i+1} + h sum X_i (from the diagonal and bit flips)."""
    state = np.asarray(state, dtype=np.complex128)
    n = int(state.size).bit_length() - 1
    out = J * zz_diag(n, periodic) * state
    idx = np.arange(1 << n, dtype=np.int64)
    for q in range(n):
        out = out + h * state[idx ^ (1 << q)]
    return out


def expval_tfim(state, J=1.0, h=0.5, periodic=False):
    """<psi|H|psi> for H = J sum Z_i Z_{i+1} + h sum X_i, in float64."""
    state = np.asarray(state, dtype=np.complex128)
    return float(np.vdot(state, apply_h_tfim(state, J, h, periodic)).real)


def qft_basis_amplitudes(n, x, ys):
    """Amplitudes <y|QFT|x> = e^{2 pi i x y / 2^n} / 2^{n/2} for the sampled
    outputs ys (closed form of the quantum Fourier transform; the phase is
    reduced exactly in integers before the float conversion)."""
    ys = np.asarray(ys, dtype=np.int64)
    frac = ((int(x) * ys) % (1 << n)).astype(np.float64) / float(1 << n)
    return np.exp(2j * np.pi * frac) / 2.0 ** (n / 2.0)


# ---------------------------------------------------------------- Kronecker checker

def kron_operator(n, G, targets, controls=()):
    """Full 2^n x 2^n operator of a gate, built from Kronecker products (n <= 10).

    U = sum_{tau,tau'} G[tau,tau'] (x)_{q=n-1..0} F_q with F_q = |tau_j><tau'_j|
    if q = targets[j], else the 2x2 identity (qubit n-1 is the leftmost
    factor, matching qubit q = bit q).  Controls: U_c = I - Pi + Pi U, with Pi
    the projector onto all controls being 1.
    """
    assert n <= 10
    G = np.asarray(G, dtype=np.complex128)
    k = len(targets)
    dim = 1 << n
    U = np.zeros((dim, dim), dtype=np.complex128)
    ket = [np.array([[1.0], [0.0]]), np.array([[0.0], [1.0]])]
    for tau in range(1 << k):
        for taup in range(1 << k):
            if G[tau, taup] == 0:
                continue
            term = np.array([[1.0 + 0j]])
            for q in range(n - 1, -1, -1):
                if q in targets:
                    j = list(targets).index(q)
                    a = (tau >> (k - 1 - j)) & 1
                    b = (taup >> (k - 1 - j)) & 1
                    f = ket[a] @ ket[b].T
                else:
                    f = np.eye(2)
                term = np.kron(term, f)
            U += G[tau, taup] * term
    if controls:
        P1 = np.array([[0.0, 0.0], [0.0, 1.0]])
        Pi = np.array([[1.0 + 0j]])
        for q in range(n - 1, -1, -1):
            Pi = np.kron(Pi, P1 if q in controls else np.eye(2))
        U = np.eye(dim) - Pi + Pi @ U
    return U


def circuit_inverse(circuit):
    """Gates of the inverse circuit: reversed order, each target block daggered."""
    inv = []
    for g in reversed(circuit):
        inv.append({"name": "UNITARY", "targets": list(g["targets"]),
                    "controls": list(g.get("controls", [])),
                    "matrix": _gates.target_matrix(g).conj().T})
    return inv
