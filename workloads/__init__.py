"""Seeded synthetic inputs shared by the oracle checks, the tests and the benchmark.

This module holds no simulation arithmetic: it only lays out circuits as
lists of gate descriptions and draws seeded random numbers (states, angles,
unitaries).  Both the oracle and the GPU path turn these descriptions into
matrices with their own code.

A gate description is a dict::

    {"name": str, "targets": [int, ...], "controls": [int, ...],
     "params": [float, ...]}            # + "matrix" (UNITARY) or "diag" (DIAG)

Names: H X Y Z SX SY SW RX RY RZ U1 CNOT CZ CU1 SWAP FSIM UNITARY DIAG.
Qubit q is bit q of the amplitude index.

The paper's benchmark circuits come from a public repository of OpenQASM
files that is not available here; the generators below are synthetic
stand-ins with the shapes the paper states (30-qubit circuits, a QFT of 480
gates at 30 qubits; benchmark-circuit table) and the configurations this
project measures.
"""
import math

import numpy as np


def gate(name, targets, controls=(), params=()):
    return {"name": name, "targets": list(targets), "controls": list(controls),
            "params": [float(p) for p in params]}


# ------------------------------------------------------------------ circuits

def qft(n):
    """Textbook quantum Fourier transform on qubits 0..n-1 (qubit n-1 = MSB).

    For j = n-1 down to 0: H(j), then for m = j-1 down to 0 a controlled
    phase U1(pi / 2^(j-m)) with control m and target j; finally SWAP(i, n-1-i)
    for i < n/2.  n + n(n-1)/2 + floor(n/2) gates (480 at 30 qubits).
    """
    c = []
    for j in range(n - 1, -1, -1):
        c.append(gate("H", [j]))
        for m in range(j - 1, -1, -1):
            c.append(gate("CU1", [j], [m], [math.pi / (1 << (j - m))]))
    for i in range(n // 2):
        c.append(gate("SWAP", [i, n - 1 - i]))
    return c


def ghz(n):
    """H on the top qubit, then a CNOT chain down to qubit 0."""
    c = [gate("H", [n - 1])]
    for q in range(n - 2, -1, -1):
        c.append(gate("CNOT", [q], [q + 1]))
    return c


def grid_shape(n):
    """rows x cols grid for n qubits: the largest divisor rows <= sqrt(n)."""
    rows = 1
    for r in range(1, int(math.isqrt(n)) + 1):
        if n % r == 0:
            rows = r
    return rows, n // rows


def supremacy(n, depth, seed=0):
    """Random supremacy-like circuit on a rows x cols grid (row-major qubits).

    Each layer: one of sqrt(X), sqrt(Y), sqrt(W) drawn uniformly per qubit;
    then one of four brick patterns (horizontal even/odd, vertical even/odd)
    drawn uniformly; each pair of the pattern gets CZ or fSim(theta, phi)
    with probability 1/2, theta and phi uniform in [0, 2 pi).  Draw order:
    layer -> qubits -> pattern -> pairs.
    """
    rng = np.random.default_rng(seed)
    rows, cols = grid_shape(n)
    names = ["SX", "SY", "SW"]
    c = []
    for _ in range(depth):
        for q in range(n):
            c.append(gate(names[int(rng.integers(3))], [q]))
        pat = int(rng.integers(4))
        pairs = []
        if pat < 2:
            for r in range(rows):
                for col in range(pat, cols - 1, 2):
                    pairs.append((r * cols + col, r * cols + col + 1))
        else:
            for r in range(pat - 2, rows - 1, 2):
                for col in range(cols):
                    pairs.append((r * cols + col, (r + 1) * cols + col))
        for a, b in pairs:
            if int(rng.integers(2)) == 0:
                c.append(gate("CZ", [b], [a]))
            else:
                th, ph = rng.uniform(0.0, 2 * math.pi, size=2)
                c.append(gate("FSIM", [a, b], [], [th, ph]))
    return c


def variational(n, layers, seed=0):
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every
    qubit, then CZ(i, (i+1) mod n) for every i; angles uniform in [0, 2 pi),
    drawn layer -> RY qubits 0..n-1 -> RZ qubits 0..n-1.
    """
    rng = np.random.default_rng(seed)
    c = []
    for _ in range(layers):
        ry = rng.uniform(0.0, 2 * math.pi, size=n)
        rz = rng.uniform(0.0, 2 * math.pi, size=n)
        for q in range(n):
            c.append(gate("RY", [q], [], [ry[q]]))
        for q in range(n):
            c.append(gate("RZ", [q], [], [rz[q]]))
        for q in range(n):
            c.append(gate("CZ", [(q + 1) % n], [q]))
    return c


def adiabatic_trotter(n, T, dt, h=1.0, periodic=True, order=2):
    """Trotterised adiabatic evolution (Sec. 3.3) as a circuit of one- and
    two-qubit gates.  H(s) = (1 - s) H0 + s H1 with H0 = -sum X_i and the
    transverse-field Ising model H1 = -sum Z_i Z_{i+1} - h sum X_i (periodic
    for n > 2), s = t / T, each step at its midpoint s_k = (k + 1/2) dt / T.
    H(s) = -a(s) sum X_i - b(s) sum Z_i Z_{i+1}, a = 1 - s + s h, b = s.

    One step of the second-order (symmetric) decomposition is
    exp(i a dt/2 sum X) exp(i b dt sum ZZ) exp(i a dt/2 sum X); first order
    drops the second half-step of X.  exp(i c X) is RX(-2c); exp(i c Z Z) is
    the diagonal gate diag(e^{ic}, e^{-ic}, e^{-ic}, e^{ic}).  Consecutive X
    half-steps of neighbouring time steps are kept as separate gates.  The
    initial state |+>^n is not part of the circuit."""
    steps = int(round(T / dt))
    pairs = [(q, q + 1) for q in range(n - 1)]
    if periodic and n > 2:
        pairs.append((n - 1, 0))
    c = []
    for k in range(steps):
        s = (k + 0.5) * dt / T
        a, b = 1.0 - s + s * h, s
        xa = a * dt / 2 if order == 2 else a * dt
        for q in range(n):
            c.append(gate("RX", [q], [], [-2.0 * xa]))
        ph = b * dt
        for i, j in pairs:
            g = gate("DIAG", [i, j])
            g["diag"] = np.exp(1j * ph * np.array([1.0, -1.0, -1.0, 1.0]))
            c.append(g)
        if order == 2:
            for q in range(n):
                c.append(gate("RX", [q], [], [-2.0 * xa]))
    return c


def parameter_slots(circuit):
    """Indices of gates that carry a trainable angle (RX/RY/RZ), in order."""
    return [i for i, g in enumerate(circuit) if g["name"] in ("RX", "RY", "RZ")]


# ------------------------------------------------------------------ states and matrices

def random_state(n, seed=0, dtype=np.complex128):
    """Random Gaussian amplitudes, normalised: re then im from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(1 << n)
    im = rng.standard_normal(1 << n)
    psi = re + 1j * im
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    return psi.astype(dtype)


def basis_index(n, seed=0):
    """Seeded basis-state index x0 in [0, 2^n)."""
    return int(np.random.default_rng(seed).integers(1 << n))


def random_unitary(k, rng):
    """Haar-random 2^k x 2^k unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def random_phases(k, rng):
    return np.exp(1j * rng.uniform(0.0, 2 * math.pi, size=1 << k))


def random_qubits(n, count, rng):
    return [int(q) for q in rng.permutation(n)[:count]]


def random_circuit(n, ngates, seed=0, kmax=3, max_controls=2):
    """Mixed gate soup for parity tests: every named kind, dense UNITARY of
    k <= kmax and DIAG gates, random (unsorted) targets and controls."""
    rng = np.random.default_rng(seed)
    one = ["H", "X", "Y", "Z", "SX", "SY", "SW", "RX", "RY", "RZ", "U1"]
    c = []
    for _ in range(ngates):
        kind = int(rng.integers(6))
        if kind == 0 and n >= 1:
            name = one[int(rng.integers(len(one)))]
            qs = random_qubits(n, 1 + min(int(rng.integers(max_controls + 1)), n - 1), rng)
            p = [float(rng.uniform(0, 2 * math.pi))] if name in ("RX", "RY", "RZ", "U1") else []
            c.append(gate(name, qs[:1], qs[1:], p))
        elif kind == 1 and n >= 2:
            name = ["SWAP", "FSIM"][int(rng.integers(2))]
            nc = min(int(rng.integers(max_controls + 1)), n - 2) if name == "SWAP" else 0
            qs = random_qubits(n, 2 + nc, rng)
            p = list(rng.uniform(0, 2 * math.pi, size=2)) if name == "FSIM" else []
            c.append(gate(name, qs[:2], qs[2:], p))
        elif kind == 2 and n >= 2:
            name = ["CNOT", "CZ", "CU1"][int(rng.integers(3))]
            qs = random_qubits(n, 2, rng)
            p = [float(rng.uniform(0, 2 * math.pi))] if name == "CU1" else []
            c.append(gate(name, qs[:1], qs[1:], p))
        elif kind == 3:
            k = 1 + int(rng.integers(min(kmax, n)))
            nc = min(int(rng.integers(max_controls + 1)), n - k)
            qs = random_qubits(n, k + nc, rng)
            g = gate("UNITARY", qs[:k], qs[k:])
            g["matrix"] = random_unitary(k, rng)
            c.append(g)
        else:
            k = 1 + int(rng.integers(min(3, n)))
            nc = min(int(rng.integers(max_controls + 1)), n - k)
            qs = random_qubits(n, k + nc, rng)
            g = gate("DIAG", qs[:k], qs[k:])
            g["diag"] = random_phases(k, rng)
            c.append(g)
    return c


def dense_windows(n, seed=0, windows=4, per=8, width=5, k=3):
    """Dense k-qubit Haar unitaries packed into `windows` disjoint windows of
    `width` adjacent qubits spread over the register, `per` gates per window
    in order: a circuit where fusing each window into one wide block pays and
    gates wider than two qubits rule out the LDS passes."""
    rng = np.random.default_rng(seed)
    starts = np.linspace(0, n - width, windows).astype(int)
    c = []
    for s in starts:
        for _ in range(per):
            qs = [int(s + q) for q in rng.choice(width, size=k, replace=False)]
            g = gate("UNITARY", qs)
            g["matrix"] = random_unitary(k, rng)
            c.append(g)
    return c
