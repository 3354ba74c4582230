"""Pins of the oracle's measurement operators (methodology section, Sec. 2:
collapse and re-normalisation, shot frequencies).  CPU only."""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import measure as OM
from oracle import statevec as S


def _ghz(n):
    return S.run_circuit(S.basis_state(n, 0), W.ghz(n))


# ------------------------------------------------------------ collapse

def test_collapse_ghz_closed_form():
    """Measuring any qubit of a GHZ state leaves |0..0> or |1..1>, each with
    probability 1/2."""
    n = 6
    psi = _ghz(n)
    for q in range(n):
        one, p1 = OM.collapse(psi, [q], 1)
        zero, p0 = OM.collapse(psi, [q], 0)
        assert abs(p1 - 0.5) <= 1e-15 and abs(p0 - 0.5) <= 1e-15
        assert np.allclose(one, S.basis_state(n, (1 << n) - 1), atol=1e-15, rtol=0)
        assert np.allclose(zero, S.basis_state(n, 0), atol=1e-15, rtol=0)


def test_collapse_projector_algebra():
    n = 7
    rng = np.random.default_rng(3)
    psi = W.random_state(n, 4)
    for r in (1, 3, 7):
        qs = [int(q) for q in rng.permutation(n)[:r]]
        total = np.zeros_like(psi)
        p_all = S.probabilities(psi, qs)
        for m in range(1 << r):
            phi, p = OM.collapse(psi, qs, m)
            # p equals the measurement probability, phi is normalised
            assert abs(p - p_all[m]) <= 1e-15
            assert abs(S.norm2(phi) - 1.0) <= 1e-14
            # P^2 = P: collapsing again changes nothing and has probability 1
            phi2, p2 = OM.collapse(phi, qs, m)
            assert abs(p2 - 1.0) <= 1e-14 and np.max(np.abs(phi2 - phi)) <= 1e-15
            # outcome m is certain afterwards, every other one impossible
            q = S.probabilities(phi, qs)
            assert abs(q[m] - 1.0) <= 1e-14 and abs(q.sum() - q[m]) <= 1e-15
            # the kept amplitudes are psi's, scaled by 1/sqrt(p)
            i = int(np.argmax(np.abs(phi)))
            assert OM.outcome_index(i, qs) == m
            total += np.sqrt(p) * phi
        # sum over outcomes of P_m psi = psi (completeness)
        assert np.max(np.abs(total - psi)) <= 1e-14


def test_collapse_onto_impossible_outcome_is_zero():
    n = 4
    phi, p = OM.collapse(S.basis_state(n, 5), [0], 0)   # |0101>: qubit 0 is 1
    assert p == 0.0 and not np.any(phi)


# ------------------------------------------------------------ inverse-CDF sampling

def test_inverse_cdf_hand_computed():
    p = np.array([0.125, 0.25, 0.375, 0.25])          # c = [0.125, 0.375, 0.75, 1.0], exact
    u = np.array([0.0, 0.124, 0.125, 0.3, 0.75, 0.999])
    assert OM.sample_inverse_cdf(p, u).tolist() == [0, 0, 1, 1, 3, 3]
    # zero-probability outcomes are never drawn
    p = np.array([0.0, 0.5, 0.0, 0.5, 0.0])
    assert OM.sample_inverse_cdf(p, np.linspace(0, 1, 101)[:-1]).tolist() == [1] * 50 + [3] * 50


def test_inverse_cdf_counts_entries_below():
    """For an increasing cumulative sum, the smallest m with x < c_m is the
    number of c_k <= x."""
    rng = np.random.default_rng(5)
    p = rng.random(64) ** 3
    u = rng.random(5000)
    c = OM.cumulative(p)
    x = u * c[-1]
    want = np.minimum((c[None, :] <= x[:, None]).sum(axis=1), 63)
    assert np.array_equal(OM.sample_inverse_cdf(p, u), want)


def test_inverse_cdf_chi_square():
    rng = np.random.default_rng(6)
    p = rng.random(16)
    p /= p.sum()
    N = 200000
    counts = np.bincount(OM.sample_inverse_cdf(p, rng.random(N)), minlength=16)
    chi2 = float(np.sum((counts - N * p) ** 2 / (N * p)))
    assert chi2 <= stats.chi2.ppf(0.999, 15)


# ------------------------------------------------------------ Metropolis frequencies

def test_metropolis_hand_computed_chain():
    # p(x=0) = 0.5: proposal 1 rejected (0.3 >= 0.25), 3 rejected (p = 0),
    # 0 accepted (0.45 < 0.5), 2 accepted (0.2 < 0.25)
    p = np.array([0.5, 0.25, 0.25, 0.0])
    counts = OM.metropolis_counts(p, [0], [[1], [3], [0], [2]], [[0.6], [0.1], [0.9], [0.4]])
    assert counts.tolist() == [3, 0, 1, 0]


def test_metropolis_limits():
    rng = np.random.default_rng(7)
    R, C, T = 32, 8, 50
    prop = rng.integers(R, size=(T, C))
    uni = rng.random((T, C))
    starts = rng.integers(R, size=C)
    # uniform p: every proposal accepted, counts = histogram of the proposals
    flat = np.full(R, 1.0 / R)
    assert np.array_equal(OM.metropolis_counts(flat, starts, prop, uni), np.bincount(prop.ravel(), minlength=R))
    # a point mass: a chain started on it never leaves
    point = np.zeros(R)
    point[9] = 1.0
    counts = OM.metropolis_counts(point, [9] * C, prop, uni)
    assert counts[9] == T * C and counts.sum() == T * C


def test_metropolis_frequencies_converge():
    rng = np.random.default_rng(8)
    R, C, T = 8, 64, 3000
    p = rng.random(R) + 0.2
    p /= p.sum()
    counts = OM.metropolis_counts(p, rng.integers(R, size=C), rng.integers(R, size=(T, C)), rng.random((T, C)))
    assert np.max(np.abs(counts / (C * T) - p)) <= 0.01
