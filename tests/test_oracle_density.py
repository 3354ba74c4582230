"""Pins of the oracle's density-matrix operators (Sec. 2: Eq. 1 applied to
density matrices).  CPU only."""
import numpy as np

import workloads as W
from oracle import density as OD
from oracle import statevec as S


def test_pure_state_evolution_matches_state_vector():
    """U |psi><psi| U^dagger = |U psi><U psi| (the state-vector oracle)."""
    n = 4
    psi = W.random_state(n, 1)
    circ = W.random_circuit(n, 30, seed=2, kmax=2, max_controls=1)
    rho = OD.run_circuit(OD.pure(psi), circ)
    assert np.max(np.abs(rho - OD.pure(S.run_circuit(psi, circ)))) <= 1e-13


def test_unitary_evolution_keeps_trace_hermiticity_and_spectrum():
    n = 3
    rng = np.random.default_rng(3)
    A = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    rho = A @ A.conj().T
    rho /= np.trace(rho)
    out = OD.run_circuit(rho, W.supremacy(n, 4, seed=5))
    assert abs(np.trace(out) - 1.0) <= 1e-14
    assert np.max(np.abs(out - out.conj().T)) <= 1e-14
    assert np.allclose(np.linalg.eigvalsh(out), np.linalg.eigvalsh(rho), atol=1e-13)


def test_channels_closed_forms():
    # full depolarizing (p = 3/4) of one qubit of a pure state leaves I/2 there
    psi = W.random_state(2, 4)
    rho = OD.apply_channel(OD.pure(psi), OD.depolarizing(0.75), target=0)
    red = np.einsum("aibi->ab", rho.reshape(2, 2, 2, 2))     # trace out qubit 0 (the low bit)
    red0 = np.einsum("iaib->ab", rho.reshape(2, 2, 2, 2))    # qubit 0's reduced state
    assert np.allclose(red0, np.eye(2) / 2, atol=1e-14)
    assert abs(np.trace(red) - 1) <= 1e-14
    # amplitude damping of |1>: probability g of |0>
    g = 0.3
    one = OD.pure(S.basis_state(1, 1))
    out = OD.apply_channel(one, OD.amplitude_damping(g), target=0)
    assert np.allclose(out, np.diag([g, 1 - g]), atol=1e-15)
    # Kraus completeness: both channels preserve the trace
    for ks in (OD.depolarizing(0.2), OD.amplitude_damping(0.6)):
        assert np.allclose(sum(K.conj().T @ K for K in ks), np.eye(2), atol=1e-15)


def test_probabilities_of_a_pure_state_match_state_vector():
    n = 5
    psi = W.random_state(n, 6)
    for qs in ([0], [4, 1], [2, 0, 3], list(range(n))):
        assert np.allclose(OD.probabilities(OD.pure(psi), qs), S.probabilities(psi, qs), atol=1e-15)


def test_flat_layout_is_row_major():
    rho = np.arange(16).reshape(4, 4).astype(complex)
    v = OD.flat(rho)
    # rho[r, c] at r * 2^n + c: column qubit q = bit q, row qubit q = bit q + n
    assert v[1 * 4 + 2] == rho[1, 2] and np.array_equal(OD.unflat(v), rho)
