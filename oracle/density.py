"""Oracle density-matrix simulation.  Test infrastructure only.

The methodology section (Sec. 2) applies Eq. 1 to state vectors and to
density matrices.  A density matrix of n qubits evolves under a gate as
rho -> U rho U^dagger and under a noise channel with Kraus operators K_k as
rho -> sum_k K_k rho K_k^dagger.  Everything here multiplies full
2^n x 2^n matrices: U is the oracle's Kronecker operator of the gate
(statevec.kron_operator), so this is only for small n.

Layout reading (the paper does not fix one): rho[r, c] is stored row-major,
at index r * 2^n + c, so in the flattened 2n-qubit vector the column's
qubit q is bit q and the row's qubit q is bit q + n.
"""
import numpy as np

from . import gates as _gates
from . import statevec as _sv


def pure(psi):
    """|psi><psi| as a 2^n x 2^n matrix."""
    psi = np.asarray(psi, dtype=np.complex128)
    return np.outer(psi, psi.conj())


def apply_gate(rho, gate):
    """U rho U^dagger with U the full operator of `gate` (controls included)."""
    n = int(rho.shape[0]).bit_length() - 1
    U = _sv.kron_operator(n, _gates.target_matrix(gate), gate["targets"], gate.get("controls", ()))
    return U @ rho @ U.conj().T


def run_circuit(rho, circuit):
    for g in circuit:
        rho = apply_gate(rho, g)
    return rho


def apply_channel(rho, kraus, target):
    """sum_k K_k rho K_k^dagger, each K_k a 2 x 2 matrix on qubit `target`."""
    n = int(rho.shape[0]).bit_length() - 1
    out = np.zeros_like(rho)
    for K in kraus:
        Kf = _sv.kron_operator(n, np.asarray(K, dtype=np.complex128), [target])
        out += Kf @ rho @ Kf.conj().T
    return out


def depolarizing(p):
    """Kraus operators of the single-qubit depolarizing channel
    rho -> (1 - p) rho + p/3 (X rho X + Y rho Y + Z rho Z)."""
    I = np.eye(2)
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1.0, -1.0])
    return [np.sqrt(1 - p) * I, np.sqrt(p / 3) * X, np.sqrt(p / 3) * Y, np.sqrt(p / 3) * Z]


def amplitude_damping(g):
    """Kraus operators of amplitude damping with decay probability g."""
    return [np.array([[1, 0], [0, np.sqrt(1 - g)]]), np.array([[0, np.sqrt(g)], [0, 0]])]


def probabilities(rho, qubits):
    """p(m) = sum of rho[i, i] over the basis states i whose measured bits
    spell m (qubits[0] = most significant bit of m), float64."""
    d = np.real(np.diag(rho)).astype(np.float64)
    n = int(d.size).bit_length() - 1
    r = len(qubits)
    out = np.zeros(1 << r)
    for i in range(d.size):
        m = 0
        for j, q in enumerate(qubits):
            m |= ((i >> q) & 1) << (r - 1 - j)
        out[m] += d[i]
    return out


def flat(rho):
    """The 2n-qubit vector of rho (row-major)."""
    return np.ascontiguousarray(rho).reshape(-1)


def unflat(v):
    N = int(round(np.sqrt(v.size)))
    return np.asarray(v).reshape(N, N)
