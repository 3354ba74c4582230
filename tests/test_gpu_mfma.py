"""GPU parity of the FP32 matrix-core block kernel (fused k = 4..6 blocks,
complex64) against the oracle and against the dense VALU kernel."""
import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import fusion as OF
from oracle import statevec as S

pytestmark = pytest.mark.gpu


def _dev(psi, dtype="c64"):
    import torch
    t = torch.complex64 if dtype == "c64" else torch.complex128
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(t).cuda()


@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("n", [11, 16])
def test_block_matches_oracle(gpu, k, n):
    rng = np.random.default_rng(10 * k + n)
    for trial in range(4):
        if trial == 0:
            qs = list(range(n - 1, n - 1 - k, -1))          # high bits: contiguous columns
        elif trial == 1:
            qs = list(range(k))                               # the lowest bits
        else:
            qs = [int(q) for q in rng.permutation(n)[:k]]     # anywhere, unsorted
        u = W.random_unitary(k, rng)
        psi0 = W.random_state(n, trial)
        st = _dev(psi0)
        qsv.qsv_apply_block(st, u, qs)
        want = S.apply_matrix(psi0, u, qs)
        err = np.max(np.abs(st.cpu().numpy() - want))
        assert err <= 1e-5, (k, n, qs, err)
        # same as the dense VALU kernel
        st2 = _dev(psi0)
        qsv.qsv_apply_matrix(st2, u, qs)
        assert np.max(np.abs(st.cpu().numpy() - st2.cpu().numpy())) <= 1e-5


def test_block_rejects_c128_and_small(gpu):
    u = W.random_unitary(4, np.random.default_rng(0))
    with pytest.raises(qsv.QsvError):
        qsv.qsv_apply_block(_dev(W.random_state(10, 0), "c128"), u, [0, 1, 2, 3])
    with pytest.raises(qsv.QsvError):
        qsv.qsv_apply_block(_dev(W.random_state(8, 0)), u, [0, 1, 2, 3])


@pytest.mark.parametrize("kmax", [4, 5, 6])
def test_greedy_mfma_plan_variational(gpu, kmax):
    """Greedy fusion into dense blocks on matrix cores (the precision +
    fusion workload shape: RY/RZ layers + CZ ring), complex64."""
    import torch
    n = 16
    circ = W.variational(n, 4, seed=3)
    psi0 = W.random_state(n, 1)
    want = S.run_circuit(psi0, circ)
    st = _dev(psi0)
    plan = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_GREEDY, kmax=kmax, use_mfma=1)
    stats = plan.stats()
    assert stats["n_mfma_blocks"] > 0
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    got = st.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - want)) <= 1e-5
    assert S.infidelity(want, got) <= 1e-6
    # block structure equals the oracle's greedy fusion
    blocks = qsv.qsv_plan_blocks(plan)
    ob = OF.greedy_blocks(circ, kmax)
    assert len(set(blocks)) == len(ob)
    for bi, members in enumerate(ob):
        assert all(blocks[g] == bi for g in members)
