"""Oracle adiabatic evolution with dense Hamiltonians.  Test infrastructure only.

Sec. 3.3 (adiabatic evolution) evolves a state under H(s) = (1 - s) H0 + s H1
from the ground state of H0 = -sum_i X_i towards that of the transverse-field
Ising model H1, either by exponentiating the full 2^n x 2^n Hamiltonian at
every time step or by a Trotter decomposition into a circuit of one- and
two-qubit gates.  The paper states neither the model's signs nor the
schedule; the readings used here:

* H1 = -sum_i Z_i Z_{i+1} - h sum_i X_i (periodic chain for n > 2, h = 1 by
  default), H0 = -sum_i X_i, linear schedule s = t / T;
* time step k covers [k dt, (k + 1) dt] and uses s at its midpoint;
* the initial state is |+>^n, the ground state of H0.

This module is the dense side: H as a matrix (qubit q = bit q) and the
step-by-step evolution psi <- expm(-i H(s_k) dt) psi with scipy's matrix
exponential, for n <= 10.
"""
import numpy as np
from scipy.linalg import expm


def pauli_sum_x(n):
    """sum_i X_i as a dense 2^n x 2^n matrix."""
    N = 1 << n
    H = np.zeros((N, N), dtype=np.complex128)
    idx = np.arange(N)
    for q in range(n):
        H[idx ^ (1 << q), idx] += 1.0
    return H


def zz_chain(n, periodic=True):
    """sum_i Z_i Z_{i+1} as a dense diagonal matrix (periodic for n > 2)."""
    N = 1 << n
    idx = np.arange(N)
    d = np.zeros(N)
    pairs = [(q, q + 1) for q in range(n - 1)]
    if periodic and n > 2:
        pairs.append((n - 1, 0))
    for a, b in pairs:
        d += np.where(((idx >> a) ^ (idx >> b)) & 1, -1.0, 1.0)
    return np.diag(d).astype(np.complex128)


def hamiltonian(n, s, h=1.0, periodic=True):
    """H(s) = (1 - s) H0 + s H1, H0 = -sum X, H1 = -sum ZZ - h sum X."""
    X = pauli_sum_x(n)
    return (1.0 - s) * (-X) + s * (-zz_chain(n, periodic) - h * X)


def plus_state(n):
    return np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)


def evolve_dense(n, T, dt, h=1.0, periodic=True, psi0=None):
    """Step-by-step exact exponentials: psi_{k+1} = expm(-i H(s_k) dt) psi_k,
    s_k = (k + 1/2) dt / T."""
    psi = plus_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128)
    steps = int(round(T / dt))
    for k in range(steps):
        s = (k + 0.5) * dt / T
        psi = expm(-1j * hamiltonian(n, s, h, periodic) * dt) @ psi
    return psi


def ground_energy(n, h=1.0, periodic=True):
    """Smallest eigenvalue of H1 (numpy's Hermitian eigensolver)."""
    return float(np.linalg.eigvalsh(hamiltonian(n, 1.0, h, periodic))[0])


def energy(psi, n, s=1.0, h=1.0, periodic=True):
    H = hamiltonian(n, s, h, periodic)
    return float(np.vdot(psi, H @ psi).real / np.vdot(psi, psi).real)
