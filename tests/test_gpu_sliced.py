"""States kept in host memory, slices processed on the device (the paper's
multi-device scheme on one re-used GPU): against the oracle, through the C
ABI."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import statevec as S

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def _host(psi, dt):
    import torch
    t = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(t).pin_memory()


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("m,a", [(10, 2), (8, 1), (11, 3), (14, 0)])
def test_sliced_matches_oracle(gpu, dt, m, a):
    n = 14
    diagonal = {"Z", "RZ", "U1", "CZ", "CU1", "DIAG"}
    # diagonal gates may touch any number of global qubits; the others at
    # most `a` global targets
    circ = [g for g in W.random_circuit(n, 150, seed=m + a, kmax=3, max_controls=2)
            if g["name"] in diagonal or sum(q >= m for q in g["targets"]) <= a]
    circ += W.supremacy(n, 3, seed=a) if a >= 2 else []
    psi0 = W.random_state(n, 1)
    want = S.run_circuit(psi0, circ)
    for mode in (qsv.PLAN_PER_GATE, qsv.PLAN_PASSES):
        st = _host(psi0, dt)
        qsv.qsv_sliced_run(st, circ, m, a, mode=mode)
        got = st.numpy().astype(np.complex128)
        assert np.max(np.abs(got - want)) <= TOL[dt], (m, a, mode)


def test_sliced_qft_with_global_controls(gpu):
    """The QFT's controlled phases between global qubits are resolved per
    group (controls dropped or the gate skipped); its final SWAPs move data
    between groups."""
    n, m = 16, 9
    psi0 = W.random_state(n, 4)
    st = _host(psi0, "c128")
    qsv.qsv_sliced_run(st, W.qft(n), m, 2, mode=qsv.PLAN_PASSES)
    assert np.max(np.abs(st.numpy() - np.fft.ifft(psi0, norm="ortho"))) <= 1e-12


def test_sliced_rejects_too_many_global_targets(gpu):
    import torch
    st = torch.zeros(1 << 12, dtype=torch.complex64).pin_memory()
    g = W.gate("UNITARY", [11, 10, 9])
    g["matrix"] = W.random_unitary(3, np.random.default_rng(0))
    with pytest.raises(qsv.QsvError):
        qsv.qsv_sliced_run(st, [g], 8, 2)


def test_sliced_qft30_closed_form(gpu):
    """A 30-qubit complex64 state in pinned host memory with 2^26-amplitude
    slices (512 MiB) and two active global qubits: sampled amplitudes of
    QFT|x> against the closed form."""
    import torch
    n = 30
    x0 = W.basis_index(n, 0)
    st = torch.zeros(1 << n, dtype=torch.complex64).pin_memory()
    st[x0] = 1.0
    qsv.qsv_sliced_run(st, W.qft(n), 26, 2, mode=qsv.PLAN_PASSES)
    ys = np.random.default_rng(3).integers(0, 1 << n, size=1 << 14)
    got = st.numpy()[ys].astype(np.complex128)
    assert np.max(np.abs(got - S.qft_basis_amplitudes(n, x0, ys))) * 2 ** (n / 2) <= 1e-4
