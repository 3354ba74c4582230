"""GPU parity of whole-circuit plans (per-gate, greedy fusion, LDS passes)
against the oracle, through the C ABI."""
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
    "random": lambda n: W.random_circuit(n, 150, seed=n, kmax=3, max_controls=2),
}


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("mode", [qsv.PLAN_PER_GATE, qsv.PLAN_GREEDY, qsv.PLAN_PASSES])
@pytest.mark.parametrize("name", sorted(CIRCUITS))
@pytest.mark.parametrize("n", [9, 12, 15])
def test_plan_matches_oracle(gpu, dt, mode, name, n):
    circ = CIRCUITS[name](n)
    psi0 = W.random_state(n, 7)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=mode, kmax=3)
    err = np.max(np.abs(got - want))
    assert err <= TOL[dt], (name, n, mode, err, stats)
    if dt == qsv.QSV_C64:
        # and the whole error vector within the FP32 rounding bound of the
        # circuit at the plan's block width (greedy blocks of 3, pass ops of 2)
        width = {qsv.PLAN_PER_GATE: 1, qsv.PLAN_GREEDY: 3, qsv.PLAN_PASSES: 2}[mode]
        assert np.linalg.norm(got - want) <= c64_bound(circ, width)


@pytest.mark.parametrize("kmax", [1, 2, 4, 5, 6])
def test_greedy_widths(gpu, kmax):
    n = 14
    circ = W.supremacy(n, 5, seed=3) + W.variational(n, 2, seed=1)
    psi0 = W.random_state(n, 2)
    want = S.run_circuit(psi0, circ)
    for dt in (qsv.QSV_C64, qsv.QSV_C128):
        got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_GREEDY, kmax=kmax, use_mfma=0)
        assert np.max(np.abs(got - want)) <= TOL[dt], (kmax, dt)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_swap_networks_in_passes(gpu, dt, seed):
    """SWAPs become relabellings in pass plans; the leftover permutation is
    moved by the bit-permutation kernel (involutions) or by SWAP kernels."""
    import torch
    n = 17
    rng = np.random.default_rng(seed)
    circ = []
    for _ in range(25):
        a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
        circ.append(W.gate("SWAP", [a, b]))
        if rng.integers(3) == 0:
            circ.append(W.gate("H", [int(rng.integers(n))]))
    if seed == 0:
        circ = [W.gate("SWAP", [i, n - 1 - i]) for i in range(n // 2)] + [W.gate("H", [3])]
    psi0 = W.random_state(n, seed)
    want = S.run_circuit(psi0, circ)
    got, stats = _run(psi0, circ, dt, mode=qsv.PLAN_PASSES)
    assert np.max(np.abs(got - want)) <= TOL[dt], stats
    # a pure permutation moves amplitudes bit-exactly
    perm_only = [g for g in circ if g["name"] == "SWAP"]
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = torch.from_numpy(psi0).to(t).cuda()
    ref = st.clone()
    plan = qsv.qsv_plan_create(n, dt, perm_only, mode=qsv.PLAN_PASSES)
    qsv.qsv_plan_execute(plan, st)
    idx = np.arange(1 << n)
    src = idx.copy()
    for g in perm_only:
        a, b = g["targets"]
        ba, bb = (src >> a) & 1, (src >> b) & 1
    # out[i] = in[perm(i)]: apply each swap to the index
    out_idx = idx.copy()
    for g in reversed(perm_only):
        a, b = g["targets"]
        ba, bb = (out_idx >> a) & 1, (out_idx >> b) & 1
        out_idx = out_idx & ~((1 << a) | (1 << b)) | (bb << a) | (ba << b)
    assert torch.equal(st.cpu(), ref.cpu()[torch.from_numpy(out_idx)])


def test_qft20_passes_c128_against_fft(gpu):
    n = 20
    psi0 = W.random_state(n, 0)
    got, stats = _run(psi0, W.qft(n), qsv.QSV_C128, mode=qsv.PLAN_PASSES)
    assert np.max(np.abs(got - np.fft.ifft(psi0, norm="ortho"))) <= 1e-12
    assert stats["n_passes"] >= 1


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_run_pass_explicit(gpu, dt):
    import torch
    n = 16
    rng = np.random.default_rng(4)
    local = [0, 1, 2, 3, 4, 5, 9, 11, 14, 15, 7, 12] + ([13] if dt == qsv.QSV_C64 else [])
    circ = []
    for _ in range(40):
        kind = rng.integers(4)
        if kind == 0:
            q = int(rng.choice(local))
            g = W.gate("UNITARY", [q])
            g["matrix"] = W.random_unitary(1, rng)
        elif kind == 1:
            a, b = [int(x) for x in rng.choice(local, 2, replace=False)]
            c = [int(x) for x in rng.choice([q for q in range(n) if q not in (a, b)], 1)]
            g = W.gate("UNITARY", [a, b], c)
            g["matrix"] = W.random_unitary(2, rng)
        elif kind == 2:
            a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
            g = W.gate("CU1", [a], [b], [rng.uniform(0, 6.28)])
        else:
            a, b = [int(x) for x in rng.choice(local, 2, replace=False)]
            g = W.gate("SWAP", [a, b])
        circ.append(g)
    psi0 = W.random_state(n, 5)
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = torch.from_numpy(psi0).to(t).cuda()
    qsv.qsv_run_pass(st, circ, local)
    want = S.run_circuit(psi0, circ)
    assert np.max(np.abs(st.cpu().numpy() - want)) <= TOL[dt]


def test_run_pass_rejects_nonlocal_target(gpu):
    import torch
    st = torch.zeros(1 << 14, dtype=torch.complex64, device="cuda")
    with pytest.raises(qsv.QsvError):
        qsv.qsv_run_pass(st, [W.gate("H", [13])], list(range(13)))
