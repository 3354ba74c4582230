"""Compiled LDS passes (plan option jit=1): parity against the oracle and
against the interpreted pass kernel, through the C ABI."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import statevec as S
from tolerance import c64_bound

pytestmark = pytest.mark.gpu

TOL = {qsv.QSV_C64: 1e-5, qsv.QSV_C128: 1e-12}


def _run(psi0, circ, dt, **kw):
    import torch
    n = int(psi0.size).bit_length() - 1
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = torch.from_numpy(psi0).to(t).cuda()
    plan = qsv.qsv_plan_create(n, dt, circ, **kw)
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    return st.cpu().numpy().astype(np.complex128), plan.stats()


CIRCUITS = {
    "qft": lambda n: W.qft(n),
    "supremacy": lambda n: W.supremacy(n, 6, seed=n),
    "variational": lambda n: W.variational(n, 3, seed=n),
    "random": lambda n: W.random_circuit(n, 150, seed=n, kmax=2, max_controls=2),
}


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("name", sorted(CIRCUITS))
@pytest.mark.parametrize("n", [9, 12, 15, 18])
def test_jit_passes_match_oracle(gpu, dt, name, n):
    circ = CIRCUITS[name](n)
    psi0 = W.random_state(n, 5)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, jit=1)
    if stats["n_passes"]:
        assert stats["n_jit_passes"] >= 1, stats
    tol = TOL[dt]
    assert np.max(np.abs(got - want)) <= tol, (name, n, stats)
    if dt == qsv.QSV_C64:
        assert np.linalg.norm(got - want) <= c64_bound(circ, 2)
    # and the interpreted kernel on the same program
    ref, _ = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, jit=0)
    assert np.max(np.abs(got - ref)) <= 2 * tol


@pytest.mark.parametrize("local_bits", [10, 11, 12, 13])
@pytest.mark.parametrize("seed", [0, 1])
def test_jit_controls_everywhere(gpu, local_bits, seed):
    """Controls on register bits, thread bits and non-local bits (the chunk
    shapes move the same qubits between the three), c64 and c128."""
    n = 16
    circ = W.random_circuit(n, 200, seed=100 + seed, kmax=2, max_controls=3)
    psi0 = W.random_state(n, seed)
    want = S.run_circuit(psi0, circ)
    for dt in (qsv.QSV_C64, qsv.QSV_C128):
        if dt == qsv.QSV_C128 and local_bits > 13:
            continue
        got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, local_bits=local_bits, jit=1)
        assert stats["n_jit_passes"] >= 1
        assert np.max(np.abs(got - want)) <= TOL[dt], (dt, local_bits, stats)
        if dt == qsv.QSV_C64:
            assert np.linalg.norm(got - want) <= c64_bound(circ, 2)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_jit_permutations_are_exact(gpu, dt):
    """X, CNOT, Toffoli and SWAP only move amplitudes: the compiled kernel
    turns their rows into register moves, so the result is bit-exact."""
    n = 15
    rng = np.random.default_rng(4)
    circ = []
    for _ in range(120):
        kind = int(rng.integers(4))
        qs = [int(q) for q in rng.choice(n, 3, replace=False)]
        if kind == 0:
            circ.append(W.gate("X", qs[:1]))
        elif kind == 1:
            circ.append(W.gate("CNOT", qs[:1], qs[1:2]))
        elif kind == 2:
            circ.append(W.gate("X", qs[:1], qs[1:3]))
        else:
            circ.append(W.gate("SWAP", qs[:2]))
    psi0 = W.random_state(n, 9)
    if dt == qsv.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, jit=1)
    assert stats["n_jit_passes"] >= 1
    assert np.array_equal(got, want)


def test_jit_qft30_sampled_against_closed_form(gpu):
    """The headline workload in the compiled configuration bench.py times:
    30-qubit QFT, complex64, default chunk (14 local bits, 512-thread
    workgroups), 2^16 sampled outputs against the closed form."""
    import torch
    n = 30
    x0 = W.basis_index(n, 0)
    st = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    st[x0] = 1.0
    plan = qsv.qsv_plan_create(n, qsv.QSV_C64, W.qft(n), mode=qsv.PLAN_PASSES, jit=1)
    assert plan.stats()["n_jit_passes"] == plan.stats()["n_launches"] == 4
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    ys = np.random.default_rng(12).integers(0, 1 << n, size=1 << 16)
    got = st[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)
    want = S.qft_basis_amplitudes(n, x0, ys)
    assert np.max(np.abs(got - want)) * 2 ** (n / 2) <= 1e-4
    assert abs(qsv.qsv_norm2(st).cpu().numpy()[0] - 1.0) <= 1e-5


def test_jit_plan_reused_and_repeated(gpu):
    """A compiled plan executes repeatedly (module loaded once) and two plans
    with the same passes share the compiled code."""
    n = 14
    circ = W.qft(n) + W.supremacy(n, 4, seed=2)
    psi0 = W.random_state(n, 3)
    want = S.run_circuit(S.run_circuit(psi0, circ), circ)
    import torch
    st = torch.from_numpy(psi0).to(torch.complex128).cuda()
    p1 = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES, jit=1)
    p2 = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES, jit=1)
    qsv.qsv_plan_execute(p1, st)
    del p1
    qsv.qsv_plan_execute(p2, st)
    torch.cuda.synchronize()
    assert np.max(np.abs(st.cpu().numpy() - want)) <= 1e-12


def _fold_circuit(n):
    circ = [W.gate("H", [q]) for q in range(3)]
    circ += [W.gate("CU1", [q + 1], [q], [0.3 * (q + 1)]) for q in range(3)]
    circ += [W.gate("X", [1], [0, 2])]
    return circ + [W.gate("SWAP", [i, n - 1 - i]) for i in range(n // 2)]


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("n", [13, 16, 19])
def test_jit_permutation_folded_into_a_pass(gpu, dt, n):
    """The final qubit reversal is stored by the pass itself (chunk pairs
    (c, sigma(c)) moved by one workgroup, in place): no permutation kernel."""
    circ = _fold_circuit(n)
    psi0 = W.random_state(n, 1)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, local_bits=12, jit=1)
    assert stats["n_launches"] == stats["n_jit_passes"] == 1, stats
    assert np.max(np.abs(got - want)) <= TOL[dt]


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_jit_folded_pure_permutation_is_exact(gpu, dt):
    n = 18
    circ = [W.gate("X", [0]), W.gate("CNOT", [2], [1])] + [W.gate("SWAP", [i, n - 1 - i]) for i in range(n // 2)]
    psi0 = W.random_state(n, 2)
    if dt == qsv.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, local_bits=12, jit=1)
    assert stats["n_launches"] == 1, stats
    assert np.array_equal(got, want)


def _cycles_circuit(n, with_gates):
    """SWAPs forming a 5-cycle and a 3-cycle of qubits (not an involution),
    with gates before, between and after them."""
    c = [W.gate("H", [q]) for q in range(4)] if with_gates else [W.gate("X", [0]), W.gate("CNOT", [2], [1])]
    for a, b in [(0, 1), (1, 7), (7, 12), (12, n - 1), (3, 9), (9, 14)]:
        c.append(W.gate("SWAP", [a, b]))
        if with_gates:
            c.append(W.gate("CU1", [a], [b], [0.1 * (a + 1)]))
    if with_gates:
        c += [W.gate("RY", [q], [], [0.2 * q]) for q in (0, 7, 9, n - 1)]
    else:
        c += [W.gate("X", [7]), W.gate("CNOT", [n - 1], [9])]
    return c


@pytest.mark.parametrize("jit", [0, 1])
@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_final_permutation_as_two_involutions(gpu, jit, dt):
    """A final relabelling that is not an involution runs as two involution
    sweeps (or folds into passes), never as a chain of SWAP gates."""
    n = 17
    circ = _cycles_circuit(n, True)
    psi0 = W.random_state(n, 3)
    want = S.run_circuit(psi0, circ)
    lb = 12 if jit else 11
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, local_bits=lb, jit=jit)
    assert stats["n_gate_ops"] == 0, stats
    assert np.max(np.abs(got - want)) <= TOL[dt], stats
    # and a pure permutation circuit stays bit-exact
    circ = _cycles_circuit(n, False)
    psi0 = W.random_state(n, 4)
    if dt == qsv.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, local_bits=lb, jit=jit)
    assert stats["n_gate_ops"] == 0, stats
    assert np.array_equal(got, S.run_circuit(psi0, circ))


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_jit_deep_supremacy_with_lookahead(gpu, dt):
    """A 20-qubit depth-16 supremacy-like circuit: later gates that commute
    with the skipped ones join open passes, at most 64 non-diagonal gates
    per pass; the result matches the oracle."""
    n = 20
    circ = W.supremacy(n, 16, seed=11)
    psi0 = W.random_state(n, 6)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, jit=1)
    assert np.max(np.abs(got - want)) <= TOL[dt], stats
    if dt == qsv.QSV_C64:
        assert np.linalg.norm(got - want) <= c64_bound(circ, 2)
    p = qsv.qsv_plan_create(n, dt, circ, mode=qsv.PLAN_PASSES, jit=1)
    order = []
    for k in range(p.stats()["n_launches"]):
        ids = qsv.qsv_plan_op_gates(p, k)
        assert sum(circ[i]["name"] != "CZ" for i in ids) <= 64
        order += ids
    assert sorted(order) == list(range(len(circ))) and order != sorted(order)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("name", sorted(CIRCUITS))
@pytest.mark.parametrize("n", [12, 16])
def test_parametric_passes_match_oracle(gpu, dt, name, n):
    """jit=2 reads matrices and angles from the program at run time: same
    results as the oracle; a second circuit of the same structure with other
    angles reuses the kernels and is right too."""
    circ = CIRCUITS[name](n)
    psi0 = W.random_state(n, 8)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES, jit=2)
    if stats["n_passes"]:
        assert stats["n_jit_passes"] >= 1, stats
    assert np.max(np.abs(got - S.run_circuit(psi0, circ))) <= TOL[dt], (name, n, stats)
    if name == "variational":
        circ2 = W.variational(n, 3, seed=n + 100)
        got2, _ = _run(psi0, circ2, dt, mode=qsv.PLAN_PASSES, jit=2)
        assert np.max(np.abs(got2 - S.run_circuit(psi0, circ2))) <= TOL[dt]
