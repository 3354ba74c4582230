"""Pins of the oracle's adiabatic evolution (Sec. 3.3: exponentiation of the
full Hamiltonian vs a Trotter decomposition into gates).  CPU only."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W
from oracle import evolution as OE
from oracle import statevec as S


def test_two_qubit_ising_ground_energy_by_hand():
    # H = -Z0 Z1 - h (X0 + X1): on (|00>+|11>)/sqrt2, (|01>+|10>)/sqrt2 it is
    # [[-1, -2h], [-2h, 1]], eigenvalues -+ sqrt(1 + 4 h^2)
    for h in (0.3, 1.0, 2.5):
        assert abs(OE.ground_energy(2, h, periodic=False) + math.sqrt(1 + 4 * h * h)) <= 1e-13


def test_driver_hamiltonian_and_plus_state():
    n = 5
    H0 = OE.hamiltonian(n, 0.0)
    assert np.allclose(np.linalg.eigvalsh(H0), np.repeat(np.arange(-n, n + 1, 2), [math.comb(n, k) for k in range(n + 1)]))
    plus = OE.plus_state(n)
    assert abs(OE.energy(plus, n, s=0.0) + n) <= 1e-13
    # |+>^n is an eigenvector of H0: exp(-i H0 t) |+> = e^{i n t} |+>
    t = 0.37
    assert np.max(np.abs(expm(-1j * H0 * t) @ plus - np.exp(1j * n * t) * plus)) <= 1e-13
    # H1 is diagonal in Z at h = 0: |0..0> has energy -(number of bonds)
    assert abs(OE.energy(S.basis_state(n, 0), n, s=1.0, h=0.0) + n) <= 1e-13


@pytest.mark.parametrize("order,ratio", [(2, 4.0), (1, 2.0)])
def test_trotter_circuit_converges_to_dense_evolution(order, ratio):
    """The gate decomposition run through the oracle's Eq. 1 approaches the
    exact exponentials with error O(dt^order)."""
    n, T = 6, 1.0
    errs = []
    for dt in (0.1, 0.05, 0.025):
        dense = OE.evolve_dense(n, T, dt)
        trot = S.run_circuit(OE.plus_state(n), W.adiabatic_trotter(n, T, dt, order=order))
        errs.append(np.linalg.norm(trot - dense))
    for a, b in zip(errs, errs[1:]):
        assert 0.7 * ratio <= a / b <= 1.3 * ratio, errs


def test_adiabatic_limit_reaches_ground_state():
    n = 6
    psi = S.run_circuit(OE.plus_state(n), W.adiabatic_trotter(n, T=20.0, dt=0.05))
    assert abs(OE.energy(psi, n) - OE.ground_energy(n)) <= 0.05
