"""Parity at the measured sizes, in the launch configuration bench.py times:
the 30-qubit QFT (complex64 and complex128, every plan) against the oracle's
closed-form amplitudes on 2^16 sampled outputs, plus properties that hold at
any size (norm, agreement between plans)."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import statevec as S

pytestmark = pytest.mark.gpu

N = 30


def _basis(n, x, dtype):
    import torch
    st = torch.zeros(1 << n, dtype=dtype, device="cuda")
    st[x] = 1.0
    return st


@pytest.mark.parametrize("dt,mode,tol", [
    (qsv.QSV_C64, qsv.PLAN_PASSES, 1e-5),
    (qsv.QSV_C64, qsv.PLAN_LEARNED, 1e-5),
    (qsv.QSV_C64, qsv.PLAN_GREEDY, 1e-5),
    (qsv.QSV_C128, qsv.PLAN_PASSES, 1e-12),
    (qsv.QSV_C128, qsv.PLAN_PER_GATE, 1e-12),
])
def test_qft30_sampled_against_closed_form(gpu, dt, mode, tol):
    import torch
    x0 = W.basis_index(N, 0)
    tdt = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = _basis(N, x0, tdt)
    plan = qsv.qsv_plan_create(N, dt, W.qft(N), mode=mode, kmax=2)
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    ys = np.random.default_rng(11).integers(0, 1 << N, size=1 << 16)
    got = st[torch.from_numpy(ys).cuda()].cpu().numpy().astype(np.complex128)
    want = S.qft_basis_amplitudes(N, x0, ys)
    err = np.max(np.abs(got - want))
    assert err <= tol
    # amplitudes are 2^-15, so also bound the error relative to that scale
    rel = err * 2 ** (N / 2)
    assert rel <= (1e-4 if dt == qsv.QSV_C64 else 1e-9), rel
    assert abs(qsv.qsv_norm2(st).cpu().numpy()[0] - 1.0) <= (1e-5 if dt == qsv.QSV_C64 else 1e-12)


def test_supremacy30_passes_equal_per_gate(gpu):
    import torch
    n = 30
    circ = W.supremacy(n, 20, seed=0)
    a = _basis(n, 0, torch.complex64)
    plan = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES)
    qsv.qsv_plan_execute(plan, a)
    b = _basis(n, 0, torch.complex64)
    plan2 = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PER_GATE)
    qsv.qsv_plan_execute(plan2, b)
    torch.cuda.synchronize()
    ov = qsv.qsv_inner(a, b).cpu().numpy()
    na = qsv.qsv_norm2(a).cpu().numpy()[0]
    nb = qsv.qsv_norm2(b).cpu().numpy()[0]
    assert abs(na - 1) <= 1e-4 and abs(nb - 1) <= 1e-4
    assert 1 - (ov[0] ** 2 + ov[1] ** 2) / (na * nb) <= 1e-6
    ys = torch.from_numpy(np.random.default_rng(1).integers(0, 1 << n, size=1 << 16)).cuda()
    assert torch.max(torch.abs(a[ys] - b[ys])).item() <= 1e-5
