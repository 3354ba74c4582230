"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the full
Kronecker-product operator (a different construction), numpy's FFT (a
library routine), closed forms, invariants, the paper's printed gate counts,
and brute force.  A few tests plant a plausible mistake in a copy of an
oracle input and check that the pin catches it.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import fusion as F
from oracle import gates as G
from oracle import mlp as M
from oracle import statevec as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ Eq. 1 vs Kronecker

def test_kron_checker_matches_numpy_kron_bit_order():
    # qubit q = bit q: on 2 qubits, a gate on qubit 0 is kron(I, G), on qubit 1 kron(G, I)
    g = W.random_unitary(1, np.random.default_rng(3))
    assert np.allclose(S.kron_operator(2, g, [0]), np.kron(np.eye(2), g), atol=0)
    assert np.allclose(S.kron_operator(2, g, [1]), np.kron(g, np.eye(2)), atol=0)
    # targets[0] is the MSB of G's index: G on targets [1, 0] of 2 qubits is G itself
    g2 = W.random_unitary(2, np.random.default_rng(4))
    assert np.allclose(S.kron_operator(2, g2, [1, 0]), g2, atol=0)
    # CNOT control 1 target 0 in the textbook |q1 q0> ordering
    cnot = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])
    assert np.allclose(S.kron_operator(2, G.X, [0], [1]), cnot, atol=0)


@pytest.mark.parametrize("seed", range(12))
def test_eq1_matches_kronecker(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 9))
    for _ in range(6):
        k = int(rng.integers(1, min(n, 4) + 1))
        c = int(rng.integers(0, min(2, n - k) + 1))
        qs = [int(q) for q in rng.permutation(n)[:k + c]]
        g = W.random_unitary(k, rng)
        psi = W.random_state(n, seed)
        got = S.apply_matrix(psi, g, qs[:k], qs[k:])
        want = S.kron_operator(n, g, qs[:k], qs[k:]) @ psi
        assert np.max(np.abs(got - want)) <= 1e-13


def test_planted_transposed_matrix_is_caught():
    # a transposed gate (wrong index order) must fail the Kronecker pin
    rng = np.random.default_rng(7)
    g = W.random_unitary(2, rng)
    psi = W.random_state(5, 1)
    wrong = S.apply_matrix(psi, g.T, [3, 1])
    want = S.kron_operator(5, g, [3, 1]) @ psi
    assert np.max(np.abs(wrong - want)) > 1e-3
    swapped_targets = S.apply_matrix(psi, g, [1, 3])
    assert np.max(np.abs(swapped_targets - want)) > 1e-3


def test_every_named_gate_matches_kronecker():
    rng = np.random.default_rng(11)
    n = 5
    circ = W.random_circuit(n, 80, seed=5)
    psi = W.random_state(n, 2)
    for g in circ:
        want = S.kron_operator(n, G.target_matrix(g), g["targets"], g["controls"]) @ psi
        got = S.apply_gate(psi, g)
        assert np.max(np.abs(got - want)) <= 1e-13
    del rng


# ------------------------------------------------------------ gate definitions

def test_gate_closed_forms():
    for name, P in (("SX", G.X), ("SY", G.Y), ("SW", G.W)):
        r = G.target_matrix({"name": name, "targets": [0], "params": []})
        assert np.allclose(r @ r, P, atol=1e-15)
    assert np.allclose(G.H @ G.H, np.eye(2), atol=1e-15)
    th = 0.731
    assert np.allclose(G.rz(th), np.exp(-0.5j * th) * G.u1(th), atol=1e-15)
    assert np.allclose(G.rx(math.pi), -1j * G.X, atol=1e-15)
    assert np.allclose(G.ry(math.pi), -1j * G.Y, atol=1e-15)
    assert np.allclose(G.fsim(0.0, 0.0), np.eye(4), atol=1e-15)
    # fSim(0, pi) = CZ; fSim(pi/2, 0) maps |01> -> -i|10>
    assert np.allclose(G.fsim(0.0, math.pi), np.diag([1, 1, 1, -1]), atol=1e-15)
    f = G.fsim(math.pi / 2, 0.0)
    assert np.allclose(f[:, 1], [0, 0, -1j, 0], atol=1e-15)
    for name in ("H", "X", "Y", "Z", "SX", "SY", "SW"):
        m = G.target_matrix({"name": name, "targets": [0], "params": []})
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-15)
    # rotation generators: d/dtheta exp(-i theta P/2) = -i/2 P exp(-i theta P/2)
    for name, fn in (("RX", G.rx), ("RY", G.ry), ("RZ", G.rz)):
        P = G.generator({"name": name})
        h = 1e-6
        d = (fn(th + h) - fn(th - h)) / (2 * h)
        assert np.allclose(d, -0.5j * P @ fn(th), atol=1e-9)


def test_swap_and_x_are_index_permutations():
    n = 6
    psi = W.random_state(n, 9)
    idx = np.arange(1 << n)
    out = S.apply_gate(psi, W.gate("SWAP", [1, 4]))
    b1, b4 = (idx >> 1) & 1, (idx >> 4) & 1
    src = idx & ~((1 << 1) | (1 << 4)) | (b4 << 1) | (b1 << 4)
    assert np.array_equal(out, psi[src])
    out = S.apply_gate(psi, W.gate("CNOT", [2], [5]))
    src = np.where((idx >> 5) & 1, idx ^ (1 << 2), idx)
    assert np.array_equal(out, psi[src])


# ------------------------------------------------------------ circuits

@pytest.mark.parametrize("n", [1, 2, 5, 10, 16])
def test_qft_equals_inverse_dft(n):
    psi = W.random_state(n, 0)
    out = S.run_circuit(psi, W.qft(n))
    assert np.max(np.abs(out - np.fft.ifft(psi, norm="ortho"))) <= 1e-12


def test_qft_basis_state_closed_form():
    n = 12
    x = W.basis_index(n, 0)
    out = S.run_circuit(S.basis_state(n, x), W.qft(n))
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / 2 ** (n / 2)
    assert np.max(np.abs(out - want)) <= 1e-13


def test_qft_closed_form_sampler_matches_eq1():
    # the sampled closed form used at 30 qubits equals the Eq. 1 run at 13
    n = 13
    x = W.basis_index(n, 4)
    full = S.run_circuit(S.basis_state(n, x), W.qft(n))
    ys = np.random.default_rng(2).integers(0, 1 << n, size=500)
    assert np.max(np.abs(S.qft_basis_amplitudes(n, x, ys) - full[ys])) <= 1e-13


def test_qft_planted_sign_error_is_caught():
    n = 8
    circ = W.qft(n)
    wrong = [dict(g, params=[-p for p in g["params"]]) if g["name"] == "CU1" else g for g in circ]
    psi = W.random_state(n, 0)
    assert np.max(np.abs(S.run_circuit(psi, wrong) - np.fft.ifft(psi, norm="ortho"))) > 1e-3


def test_ghz_and_bell():
    for n in (2, 3, 9):
        out = S.run_circuit(S.basis_state(n, 0), W.ghz(n))
        want = np.zeros(1 << n, dtype=np.complex128)
        want[0] = want[-1] = 1 / math.sqrt(2)
        assert np.max(np.abs(out - want)) <= 1e-15


@pytest.mark.parametrize("maker", ["random", "supremacy", "variational"])
def test_norm_and_inverse(maker):
    n = 9
    circ = {"random": lambda: W.random_circuit(n, 60, seed=3),
            "supremacy": lambda: W.supremacy(n, 6, seed=1),
            "variational": lambda: W.variational(n, 3, seed=2)}[maker]()
    psi = W.random_state(n, 4)
    out = S.run_circuit(psi, circ)
    assert abs(S.norm2(out) - 1.0) <= 1e-13
    back = S.run_circuit(out, S.circuit_inverse(circ))
    assert np.max(np.abs(back - psi)) <= 1e-13


def test_generator_gate_counts():
    assert len(W.qft(30)) == 480 and len(W.qft(20)) == 220 and len(W.qft(33)) == 577
    assert len(W.variational(32, 40)) == 3840
    c4 = W.variational(24, 12)
    assert len(c4) == 864 and len(W.parameter_slots(c4)) == 576
    assert W.grid_shape(30) == (5, 6) and W.grid_shape(33) == (3, 11)


# ------------------------------------------------------------ reductions

def test_probabilities():
    n = 7
    ghz = S.run_circuit(S.basis_state(n, 0), W.ghz(n))
    p = S.probabilities(ghz, [6, 3])
    assert np.allclose(p, [0.5, 0, 0, 0.5], atol=1e-15)
    # a basis state puts all weight on its bits, qubits[0] as the MSB
    x = 0b1011001
    p = S.probabilities(S.basis_state(n, x), [0, 3, 4])
    assert p.argmax() == (1 << 2) | (1 << 1) | 1 and p.max() == 1.0
    psi = W.random_state(n, 5)
    assert abs(S.probabilities(psi, [2]).sum() - 1) <= 1e-14
    full = S.probabilities(psi, list(range(n - 1, -1, -1)))
    assert np.allclose(full, np.abs(psi) ** 2, atol=1e-16, rtol=1e-14)
    # brute force marginal
    q = [5, 1]
    bf = np.zeros(4)
    for i in range(1 << n):
        bf[((i >> 5) & 1) * 2 + ((i >> 1) & 1)] += abs(psi[i]) ** 2
    assert np.allclose(S.probabilities(psi, q), bf, atol=1e-16, rtol=1e-13)


def test_tfim_energy():
    n = 6
    zero = S.basis_state(n, 0)
    assert abs(S.expval_tfim(zero, 1.0, 0.5) - (n - 1)) <= 1e-14
    assert abs(S.expval_tfim(zero, 1.0, 0.5, periodic=True) - n) <= 1e-14
    plus = S.run_circuit(zero, [W.gate("H", [q]) for q in range(n)])
    assert abs(S.expval_tfim(plus, 1.0, 0.5) - 0.5 * n) <= 1e-14
    # dense operator from Kronecker products
    psi = W.random_state(n, 8)
    Hm = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for i in range(n - 1):
        Hm += S.kron_operator(n, np.kron(G.Z, G.Z), [i + 1, i])
    for i in range(n):
        Hm += 0.5 * S.kron_operator(n, G.X, [i])
    assert abs(S.expval_tfim(psi) - np.vdot(psi, Hm @ psi).real) <= 1e-13


def test_infidelity():
    psi = W.random_state(6, 1)
    assert abs(S.infidelity(psi, psi * np.exp(0.3j))) <= 1e-15
    phi = W.random_state(6, 2)
    want = 1 - abs(np.vdot(psi, phi)) ** 2
    assert abs(S.infidelity(psi, phi) - want) <= 1e-15
    # unnormalised inputs: the norms divide out (hand-computed cases)
    assert S.infidelity(np.array([1.0, 0.0]), np.array([1.0, 1.0])) == 0.5
    assert S.infidelity(np.array([2.0, 0.0]), np.array([0.0, 3.0j])) == 1.0
    assert abs(S.infidelity(np.array([1.0, 1.0j]), np.array([3.0, 3.0j]))) <= 1e-15
    assert abs(S.infidelity(3.0 * psi, 0.5 * phi) - want) <= 1e-14


# ------------------------------------------------------------ fusion (Sec. 3.2)

def _golden_qft():
    with open(os.path.join(GOLDEN, "benchmark_circuits_qft30.txt")) as f:
        for line in f:
            if line.startswith("qft"):
                _, d, g, df, gf = line.split()
                return int(d), int(g), int(df), int(gf)


def test_fusion_counts_match_paper_table():
    depth, gates, depth_f, gates_f = _golden_qft()
    c = W.qft(30)
    assert len(c) == gates
    assert F.depth([F.qubits_of(g) for g in c]) == depth
    blocks = F.greedy_blocks(c, kmax=2)
    assert len(blocks) == gates_f
    assert F.depth([F.block_qubits(c, m) for m in blocks]) == depth_f


@pytest.mark.parametrize("kmax", [2, 3, 5])
def test_fused_circuit_equals_unfused(kmax):
    n = 8
    for circ in (W.qft(n), W.supremacy(n, 5, seed=2), W.random_circuit(n, 50, seed=9, kmax=2)):
        blocks = F.greedy_blocks(circ, kmax)
        assert sorted(i for b in blocks for i in b) == list(range(len(circ)))
        assert all(len(F.block_qubits(circ, b)) <= max(kmax, len(F.qubits_of(circ[b[0]]))) for b in blocks)
        psi = W.random_state(n, 3)
        a = S.run_circuit(psi, circ)
        b = S.run_circuit(psi, F.fused_circuit(circ, kmax))
        assert np.max(np.abs(a - b)) <= 1e-13


# ------------------------------------------------------------ gradients

def test_param_shift_matches_finite_differences_and_adjoint():
    n = 5
    circ = W.variational(n, 2, seed=4)
    ps = A.grad_param_shift(circ, n)
    fd = A.grad_fd(circ, n, step=1e-5)
    e, adj = A.grad_adjoint(circ, n)
    assert abs(e - A.expval(circ, n)) <= 1e-13
    assert np.max(np.abs(ps - fd)) <= 1e-8
    assert np.max(np.abs(adj - ps)) <= 1e-12


def test_planted_adjoint_sign_error_is_caught():
    n = 4
    circ = W.variational(n, 1, seed=1)
    ps = A.grad_param_shift(circ, n)
    _, adj = A.grad_adjoint(circ, n)
    assert np.max(np.abs(-adj - ps)) > 1e-3


# ------------------------------------------------------------ MLP

def _mlp(rng, sizes):
    return [(rng.standard_normal((a, b)) / math.sqrt(a), 0.1 * rng.standard_normal(b))
            for a, b in zip(sizes[:-1], sizes[1:])]


def test_mlp_forward_hand_computed():
    """A 2 -> 2 -> 1 network evaluated by hand: ReLU on the hidden layer only,
    x @ W with W stored [fan_in, fan_out]."""
    params = [(np.array([[1.0, -2.0], [3.0, 1.0]]), np.array([0.5, -1.0])),
              (np.array([[2.0], [-1.0]]), np.array([0.25]))]
    X = np.array([[1.0, 1.0], [2.0, -1.0], [-1.0, 0.0]])
    # row 1: hidden [4.5, -2] -> [4.5, 0] -> 9 + 0.25
    # row 2: hidden [-0.5, -6] -> [0, 0] -> 0.25
    # row 3: hidden [-0.5, 1] -> [0, 1] -> -1 + 0.25 (a negative output: no ReLU on it)
    pred, (acts, pre) = M.forward(params, X)
    assert np.array_equal(pred, [9.25, 0.25, -0.75])
    assert np.array_equal(pre[0], [[4.5, -2.0], [-0.5, -6.0], [-0.5, 1.0]])
    assert np.array_equal(acts[1], [[4.5, 0.0], [0.0, 0.0], [0.0, 1.0]])
    assert M.mse(pred, np.array([9.25, 1.25, 0.25])) == 2.0 / 3.0


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = _mlp(rng, [5, 7, 6, 1])
    X = rng.standard_normal((9, 5))
    t = rng.standard_normal(9)
    pred, cache = M.forward(params, X)
    grads = M.backward(params, cache, pred, t)
    h = 1e-6
    for li, (Wl, bl) in enumerate(params):
        for arr, garr in ((Wl, grads[li][0]), (bl, grads[li][1])):
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = M.mse(M.forward(params, X)[0], t)
                arr[idx] = old - h
                lm = M.mse(M.forward(params, X)[0], t)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - garr[idx]) <= 1e-6


def test_adam_first_step_closed_form():
    # after one step with zero moments, mhat = g and vhat = g^2: step = lr * g/(|g|+eps)
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_golden_adjoint24_routes_agree():
    """The stored 24-qubit gradients (tests/golden/adjoint24_cfg4.txt, written
    by the oracle): on the seeded subset the oracle's adjoint equals its
    parameter shift (exact for rotation gates, Sec. 3.4) to rounding, and
    central finite differences with step 1e-5 agree to O(h^2); every one of
    the 576 angles has an entry and the energy lies in [-E_max, E_max]."""
    path = os.path.join(os.path.dirname(__file__), "golden", "adjoint24_cfg4.txt")
    energy, adj, sub = None, {}, {}
    for line in open(path):
        if line.startswith("# energy"):
            energy = float(line.split()[2])
        elif line.startswith("adjoint "):
            _, i, g = line.split()
            adj[int(i)] = float(g)
        elif line.startswith("subset "):
            _, i, ps, fd = line.split()
            sub[int(i)] = (float(ps), float(fd))
    assert sorted(adj) == list(range(576)) and len(sub) == 32
    # |<H>| <= 23 bonds + 0.5 * 24 fields
    assert energy is not None and abs(energy) <= 23 + 12
    idx = sorted(sub)
    a = np.array([adj[i] for i in idx])
    ps = np.array([sub[i][0] for i in idx])
    fd = np.array([sub[i][1] for i in idx])
    assert np.max(np.abs(a - ps)) <= 1e-12
    assert np.max(np.abs(fd - ps)) <= 1e-8
