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


@pytest.mark.parametrize("dt,mode,jit,tol", [
    (qsv.QSV_C64, qsv.PLAN_PASSES, 0, 1e-5),
    (qsv.QSV_C64, qsv.PLAN_PASSES, 1, 1e-5),
    (qsv.QSV_C64, qsv.PLAN_LEARNED, 1, 1e-5),
    (qsv.QSV_C64, qsv.PLAN_GREEDY, 0, 1e-5),
    (qsv.QSV_C128, qsv.PLAN_PASSES, 0, 1e-12),
    (qsv.QSV_C128, qsv.PLAN_PASSES, 1, 1e-12),
    (qsv.QSV_C128, qsv.PLAN_PER_GATE, 0, 1e-12),
])
def test_qft30_sampled_against_closed_form(gpu, dt, mode, jit, tol):
    """The learned case loads the shipped cost model (the headline's plan
    choice), so it runs whichever plan the network picks."""
    import os
    import torch
    x0 = W.basis_index(N, 0)
    tdt = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = _basis(N, x0, tdt)
    if mode == qsv.PLAN_LEARNED:
        from paper_2203_08826_amd import cost_model as CM
        assert os.path.exists(CM.DEFAULT_PATH)
        CM.load_into_library(CM.DEFAULT_PATH)
    try:
        plan = qsv.qsv_plan_create(N, dt, W.qft(N), mode=mode, kmax=2, jit=jit)
    finally:
        if mode == qsv.PLAN_LEARNED:
            qsv.qsv_cost_model_clear()
    if mode == qsv.PLAN_LEARNED:
        assert plan.stats()["predicted_s"] > 0
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


# ------------------------------------------------------------ sampled groups at full size
#
# A gate (Eq. 1) acts on each group -- the 2^k amplitudes that differ only in
# the target bits, with every control bit set -- independently.  At 30-32
# qubits the oracle applies the gate to sampled groups: their amplitudes are
# gathered before the launch and compared with the same groups after it.

def _groups(n, targets, controls, count, rng):
    """[count, 2^k] amplitude indices of random groups, member tau at column
    tau (targets[0] = most significant bit of tau)."""
    k = len(targets)
    base = rng.integers(0, 1 << n, size=count, dtype=np.int64)
    for q in targets:
        base &= ~(1 << q)
    for q in controls:
        base |= 1 << q
    tau = np.arange(1 << k, dtype=np.int64)
    off = np.zeros(1 << k, dtype=np.int64)
    for j, q in enumerate(targets):
        off |= ((tau >> (k - 1 - j)) & 1) << q
    return base[:, None] | off[None, :]


def _oracle_groups(G, x):
    """Eq. 1 on every group: the groups stacked as the high bits of a
    (log2 count + k)-qubit state whose low k bits are the targets."""
    cnt, d = x.shape
    k = d.bit_length() - 1
    flat = S.apply_matrix(x.reshape(-1), G, list(range(k - 1, -1, -1)))
    return flat.reshape(cnt, d)


def _block_bound(k, u, gauss=False):
    """Worst-case 2-norm error of one k-qubit block applied in floating point
    with unit roundoff u, relative to the group's norm (m = 2^k, G unitary).

    Complex products, or the real-GEMM form of the matrix cores (2m-term real
    dot products): (4 m sqrt(m) + sqrt(m) + 1) u.

    Gauss's three-product form (Yr = T1 - T2, Yi = T3 - T1 - T2 with
    T3 = (Gr + Gi)(Xr + Xi), the sums rounded): componentwise the imaginary
    part errs by at most (m + 4) u [(|Gr| + |Gi|)(|Xr| + |Xi|) + |Gr||Xr| +
    |Gi||Xi|] (Higham 1992), the real part by m u (|Gr||Xr| + |Gi||Xi|) plus
    one rounding.  With |Gr| + |Gi| <= sqrt(2) |G| entrywise, ||G||_F =
    sqrt(m) and || |Xr| + |Xi| || <= sqrt(2) ||x||, the two bracketed terms
    are at most 2 sqrt(m) and sqrt(2 m) times ||x||: in all
    (5 (m + 4) sqrt(m) + 1) u."""
    m = 2 ** k
    if gauss:
        return (5 * (m + 4) * np.sqrt(m) + 1) * u
    return (4 * m * np.sqrt(m) + np.sqrt(m) + 1) * u


def _check_groups(st, n, G, targets, controls, apply, rng, count=4096, gauss=False):
    import torch
    idx = _groups(n, targets, controls, count, rng)
    di = torch.from_numpy(idx.reshape(-1)).cuda()
    x = st[di].cpu().numpy().astype(np.complex128).reshape(idx.shape)
    # a sample of amplitudes outside the groups (a control bit 0) stays put
    if controls:
        free = rng.integers(0, 1 << n, size=count, dtype=np.int64) & ~(1 << controls[0])
        dfree = torch.from_numpy(free).cuda()
        before = st[dfree].clone()
    apply(st)
    torch.cuda.synchronize()
    y = st[di].cpu().numpy().astype(np.complex128).reshape(idx.shape)
    want = _oracle_groups(np.asarray(G, dtype=np.complex128), x)
    rel = np.linalg.norm(y - want, axis=1) / np.linalg.norm(x, axis=1)
    u = 2.0 ** -24 if st.dtype == torch.complex64 else 2.0 ** -53
    assert np.max(rel) <= _block_bound(len(targets), u, gauss), np.max(rel)
    if controls:
        assert torch.equal(st[dfree], before)
    return float(np.max(rel))


@pytest.mark.parametrize("n", [30, 32])
@pytest.mark.parametrize("k", [4, 5, 6])
def test_mfma_block_full_size_sampled_groups(gpu, n, k):
    import torch
    rng = np.random.default_rng(1000 + 10 * n + k)
    g = torch.Generator(device="cuda").manual_seed(n + k)
    st = torch.randn(1 << n, dtype=torch.complex64, device="cuda", generator=g)
    for qs in (list(range(n - 1, n - 1 - k, -1)), list(range(k)), [int(q) for q in rng.permutation(n)[:k]]):
        u = W.random_unitary(k, rng)
        # k = 5, 6 run Gauss's three-product form on the matrix cores
        _check_groups(st, n, u, qs, [], lambda s: qsv.qsv_apply_block(s, u, qs), rng, gauss=k >= 5)
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt,n", [("c64", 30), ("c64", 33), ("c128", 30)])
def test_gate_kernels_full_size_sampled_groups(gpu, dt, n):
    """Dense, controlled and two-qubit gates on low, middle and high qubits,
    with the launch shapes of full-size states (one unit per thread, the
    shuffle path on low qubits, grid-stride rounds at 33 qubits)."""
    import torch
    rng = np.random.default_rng(2000 + n)
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    g = torch.Generator(device="cuda").manual_seed(n)
    st = torch.randn(1 << n, dtype=tdt, device="cuda", generator=g)
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    cases = [(H, [0], []), (H, [3], []), (H, [12], []), (H, [n - 8], []), (H, [n - 1], []),
             (W.random_unitary(1, rng), [n - 2], [5]),
             (W.random_unitary(2, rng), [n - 1, 3], []),
             (W.random_unitary(2, rng), [n - 3, n - 5], [0]),
             (W.random_unitary(3, rng), [1, n - 1, 17], [])]
    for G, tg, cs in cases:
        _check_groups(st, n, G, tg, cs, lambda s: qsv.qsv_apply_matrix(s, G, tg, cs), rng)
    # fSim through its own entry point
    th, ph = 0.7, 1.9
    F = np.array([[1, 0, 0, 0], [0, np.cos(th), -1j * np.sin(th), 0], [0, -1j * np.sin(th), np.cos(th), 0],
                  [0, 0, 0, np.exp(-1j * ph)]])
    _check_groups(st, n, F, [n - 1, 10], [], lambda s: qsv.qsv_apply_fsim(s, n - 1, 10, th, ph), rng)
    del st
    torch.cuda.empty_cache()
