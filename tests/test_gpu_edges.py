"""Degenerate sizes through the C ABI: states of one to three qubits (a single
group, fewer amplitudes than a wave) under every plan kind and the
per-gate entry points, gates on every qubit of the register, empty
circuits, and the reductions and measurement calls on the smallest states,
each against the oracle (Eq. 1; the measurement operators of Sec. 2)."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import measure as OM
from oracle import statevec as S

pytestmark = pytest.mark.gpu

TOL = {qsv.QSV_C64: 1e-5, qsv.QSV_C128: 1e-12}


def _dev(psi, dt):
    import torch
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(t).cuda().contiguous()


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


PLANS = [dict(mode=qsv.PLAN_PER_GATE), dict(mode=qsv.PLAN_GREEDY, kmax=1), dict(mode=qsv.PLAN_GREEDY, kmax=2),
         dict(mode=qsv.PLAN_GREEDY, kmax=3, use_mfma=1), dict(mode=qsv.PLAN_PASSES, jit=0),
         dict(mode=qsv.PLAN_PASSES, jit=1), dict(mode=qsv.PLAN_LEARNED)]


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_states_every_plan(gpu, dt, n):
    circ = W.random_circuit(n, 40, seed=10 + n, kmax=n, max_controls=min(2, n - 1))
    psi0 = W.random_state(n, 5)
    want = S.run_circuit(psi0, circ)
    for kw in PLANS:
        try:
            plan = qsv.qsv_plan_create(n, dt, circ, **kw)
        except qsv.QsvError:
            assert kw.get("kmax", 0) > n, kw   # only a block wider than the register is refused
            continue
        st = _dev(psi0, dt)
        qsv.qsv_plan_execute(plan, st)
        assert np.max(np.abs(_host(st) - want)) <= TOL[dt], (n, kw)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_empty_circuit_leaves_the_state(gpu, dt):
    import torch
    psi0 = W.random_state(5, 2)
    st = _dev(psi0, dt)
    ref = st.clone()
    for kw in PLANS:
        plan = qsv.qsv_plan_create(5, dt, [], **kw)
        assert plan.stats()["n_launches"] == 0
        qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    assert torch.equal(st, ref)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("k", [1, 4, 6])
def test_gate_on_every_qubit(gpu, dt, k):
    """A dense gate whose targets are the whole register (one group)."""
    rng = np.random.default_rng(k)
    u = W.random_unitary(k, rng)
    targets = [int(q) for q in rng.permutation(k)]
    g = W.gate("UNITARY", targets)
    g["matrix"] = u
    psi0 = W.random_state(k, 3)
    st = _dev(psi0, dt)
    qsv.qsv_apply_matrix(st, u, targets)
    assert np.max(np.abs(_host(st) - S.apply_gate(psi0, g))) <= TOL[dt]


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_reductions_and_measurement_on_one_and_two_qubits(gpu, dt):
    import torch
    for n in (1, 2):
        psi = W.random_state(n, 8)
        st = _dev(psi, dt)
        tol = 1e-6 if dt == qsv.QSV_C64 else 1e-13
        assert abs(float(qsv.qsv_norm2(st).item()) - 1.0) <= tol
        for qs in ([0], [n - 1], list(range(n))[::-1]):
            p = qsv.qsv_probabilities(st, qs).cpu().numpy()
            assert np.max(np.abs(p - S.probabilities(psi, qs))) <= tol, (n, qs)
        e = float(qsv.qsv_expval_zz_x(st, 1.0, 0.5).item())
        assert abs(e - S.expval_tfim(psi, 1.0, 0.5, False)) <= tol
        # collapse onto outcome 1 of the top qubit
        pr = float(qsv.qsv_collapse(st, [n - 1], 1).item())
        want, pw = OM.collapse(psi, [n - 1], 1)
        assert abs(pr - pw) <= tol
        assert np.max(np.abs(_host(st) - want)) <= (1e-5 if dt == qsv.QSV_C64 else 1e-12)
    # sampling from two outcomes
    probs = torch.tensor([0.25, 0.75], dtype=torch.float64, device="cuda")
    u = torch.tensor([0.0, 0.2, 0.25, 0.3, 0.999], dtype=torch.float64, device="cuda")
    _, smp, cnt = qsv.qsv_sample_cdf(probs, u)
    assert smp.cpu().tolist() == [0, 0, 1, 1, 1]
    assert cnt.cpu().numpy().astype(np.int64).tolist() == [2, 3]
