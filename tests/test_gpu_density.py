"""Density matrices on the GPU (Eq. 1 applied as rho -> G rho G^dagger;
Kraus channels; trace and diagonal probabilities) against the oracle's full
operators, through the C ABI."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import density as OD
from oracle import statevec as S

pytestmark = pytest.mark.gpu

TOL = {qsv.QSV_C64: 1e-5, qsv.QSV_C128: 1e-12}


def _dev(rho, dt):
    import torch
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    return torch.from_numpy(OD.flat(rho)).to(t).cuda().contiguous()


def _mixed(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("n", [2, 4, 6])
def test_dm_circuit_matches_oracle(gpu, dt, n):
    import torch
    rho0 = _mixed(n, n)
    if dt == qsv.QSV_C64:
        rho0 = rho0.astype(np.complex64).astype(np.complex128)
    circ = W.random_circuit(n, 40, seed=n, kmax=min(n, 3), max_controls=1) + W.supremacy(n, 2, seed=n)
    want = OD.run_circuit(rho0, circ)
    for kw in (dict(mode=qsv.PLAN_PER_GATE), dict(mode=qsv.PLAN_GREEDY, kmax=3),
               dict(mode=qsv.PLAN_PASSES, jit=0), dict(mode=qsv.PLAN_PASSES, jit=1)):
        if kw["mode"] == qsv.PLAN_PASSES and 2 * n < 9:
            continue
        st = _dev(rho0, dt)
        plan = qsv.qsv_dm_plan_create(n, dt, circ, **kw)
        qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        got = OD.unflat(st.cpu().numpy().astype(np.complex128))
        assert np.max(np.abs(got - want)) <= TOL[dt], (n, kw)
        assert np.max(np.abs(got - got.conj().T)) <= 2 * TOL[dt]
        tr = qsv.qsv_dm_trace(st).cpu().numpy()
        assert abs(tr[0] - 1.0) <= (1e-5 if dt == qsv.QSV_C64 else 1e-12) and abs(tr[1]) <= 1e-6


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_channels_and_probabilities(gpu, dt):
    import torch
    n = 5
    rho = _mixed(n, 11)
    if dt == qsv.QSV_C64:
        rho = rho.astype(np.complex64).astype(np.complex128)
    st = _dev(rho, dt)
    for kraus, q in ((OD.depolarizing(0.3), 2), (OD.amplitude_damping(0.45), 0), (OD.depolarizing(0.75), 4)):
        qsv.qsv_dm_apply_channel(st, kraus, q)
        rho = OD.apply_channel(rho, kraus, q)
    torch.cuda.synchronize()
    got = OD.unflat(st.cpu().numpy().astype(np.complex128))
    assert np.max(np.abs(got - rho)) <= TOL[dt]
    for qs in ([0], [4, 1], [3, 0, 2], list(range(n))):
        p = qsv.qsv_dm_probabilities(st, qs).cpu().numpy()
        assert np.max(np.abs(p - OD.probabilities(got, qs))) <= 1e-14 * (1 << n)


def test_dm_pure_state_at_12_qubits(gpu):
    """rho0 = |psi><psi| of 12 qubits (a 24-qubit vector, 128 MiB): after a
    circuit through compiled passes the sampled entries equal
    psi'[r] conj(psi'[c]) with psi' the state-vector oracle's result."""
    import torch
    n = 12
    psi = W.random_state(n, 3)
    circ = W.supremacy(n, 6, seed=9) + W.qft(n)
    d = torch.from_numpy(psi).cuda()
    st = (d[:, None] * d.conj()[None, :]).reshape(-1).contiguous()
    plan = qsv.qsv_dm_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES, jit=1)
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    out = S.run_circuit(psi, circ)
    rng = np.random.default_rng(4)
    r = rng.integers(1 << n, size=4096)
    c = rng.integers(1 << n, size=4096)
    got = st[torch.from_numpy(r * (1 << n) + c).cuda()].cpu().numpy()
    assert np.max(np.abs(got - out[r] * out[c].conj())) <= 1e-12
    p = qsv.qsv_dm_probabilities(st, [11, 0, 5]).cpu().numpy()
    assert np.max(np.abs(p - S.probabilities(out, [11, 0, 5]))) <= 1e-12
