"""Trotterised adiabatic evolution (Sec. 3.3) on the GPU: the gate circuit
through every plan kind against the oracle's run of the same circuit, and
against the oracle's dense-Hamiltonian evolution within the Trotter error."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import evolution as OE
from oracle import statevec as S

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
    return st.cpu().numpy().astype(np.complex128), st


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("n", [8, 14])
def test_trotter_circuit_matches_oracle(gpu, dt, n):
    circ = W.adiabatic_trotter(n, T=2.0, dt=0.1)
    psi0 = OE.plus_state(n)
    want = S.run_circuit(psi0, circ)
    for kw in (dict(mode=qsv.PLAN_PER_GATE), dict(mode=qsv.PLAN_GREEDY, kmax=2),
               dict(mode=qsv.PLAN_PASSES, jit=0), dict(mode=qsv.PLAN_PASSES, jit=1)):
        got, _ = _run(psi0, circ, dt, **kw)
        assert np.max(np.abs(got - want)) <= TOL[dt], (n, kw)


def test_trotter_against_dense_exponentials(gpu):
    """At 8 qubits the GPU's Trotter state is within the oracle's Trotter
    error (measured against its dense evolution) of the exact evolution, and
    its energy under H1 follows the adiabatic path."""
    import torch
    n, T, step = 8, 4.0, 0.05
    circ = W.adiabatic_trotter(n, T=T, dt=step)
    dense = OE.evolve_dense(n, T, step)
    trot_err = np.linalg.norm(S.run_circuit(OE.plus_state(n), circ) - dense)
    got, st = _run(OE.plus_state(n), circ, qsv.QSV_C128, mode=qsv.PLAN_PASSES, jit=1)
    assert np.linalg.norm(got - dense) <= trot_err + 1e-11
    # <H1> = -(sum ZZ + sum X) through the library's reduction (periodic chain)
    e = float(qsv.qsv_expval_zz_x(st, J=-1.0, h=-1.0, periodic=True).cpu().numpy()[0])
    assert abs(e - OE.energy(dense, n)) <= 2 * trot_err * np.linalg.norm(OE.hamiltonian(n, 1.0), 2) + 1e-9
