"""Measurement probabilities (methodology section, measurement operator) for
every number of measured qubits r = 1..n, through the C ABI.

Small and medium n: every r against the oracle on a random state.  At 30
qubits (complex64, 8 GiB state) every r against closed forms: a basis state
(one outcome with probability exactly 1), a GHZ state (two outcomes, each
exactly the square of the stored amplitude), a product state (each outcome a
product of per-qubit factors), plus brute-force sums over the stored
amplitudes of a random state for sampled outcomes.
"""
import math

import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import statevec as S

pytestmark = pytest.mark.gpu


def _dev(psi, dt):
    import torch
    t = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(t).cuda().contiguous()


def _as_stored(psi, dt):
    return np.asarray(psi, dtype=np.complex64 if dt == "c64" else np.complex128).astype(np.complex128)


def _qubit_orders(n, r, rng):
    """Measured qubit lists of length r: a random subset in random order, the
    lowest r ascending and the highest r descending (natural outcome order)."""
    return [[int(q) for q in rng.permutation(n)[:r]], list(range(r)), list(range(n - 1, n - 1 - r, -1))]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 5, 7, 13, 20])
def test_every_r_matches_oracle(gpu, dt, n):
    rng = np.random.default_rng(100 + n)
    psi = _as_stored(W.random_state(n, 3), dt)
    d = _dev(psi, dt)
    for r in range(1, n + 1):
        for qs in _qubit_orders(n, r, rng):
            got = qsv.qsv_probabilities(d, qs).cpu().numpy()
            want = S.probabilities(psi, qs)
            # both sides sum 2^(n-r) non-negative float64 terms in different
            # orders: each within (2^(n-r) - 1) 2^-53 of the exact sum (<= 1)
            assert np.max(np.abs(got - want)) <= 2.0 ** (n - r + 1 - 53) + 1e-16, (n, r, qs)
            # fixed summation order: the same bits on a second call
            assert np.array_equal(qsv.qsv_probabilities(d, qs).cpu().numpy(), got)


def _outcome_bits(m, qs):
    """Values of the measured qubits for outcome m (qs[0] = MSB of m)."""
    r = len(qs)
    return [(m >> (r - 1 - j)) & 1 for j in range(r)]


def test_every_r_closed_forms_30q(gpu):
    import torch
    n = 30
    rng = np.random.default_rng(7)
    N = 1 << n
    # basis state |x>
    x = int(rng.integers(N))
    st = torch.zeros(N, dtype=torch.complex64, device="cuda")
    st[x] = 1.0
    for r in range(1, n + 1):
        qs = _qubit_orders(n, r, rng)[r % 3]
        p = qsv.qsv_probabilities(st, qs)
        mx = sum(((x >> q) & 1) << (r - 1 - j) for j, q in enumerate(qs))
        assert int(torch.count_nonzero(p).item()) == 1, r
        assert float(p[mx].item()) == 1.0, (r, qs)
        del p
    # GHZ: amplitude a at |0..0> and |1..1>
    st.zero_()
    a = np.float32(1 / math.sqrt(2))
    st[0] = complex(a)
    st[N - 1] = complex(a)
    a2 = float(a) * float(a)   # exact in float64
    for r in range(1, n + 1):
        qs = _qubit_orders(n, r, rng)[(r + 1) % 3]
        p = qsv.qsv_probabilities(st, qs)
        assert int(torch.count_nonzero(p).item()) == 2, r
        assert float(p[0].item()) == a2 and float(p[(1 << r) - 1].item()) == a2, (r, qs)
        del p
    del st
    torch.cuda.empty_cache()
    # product state: qubit q holds cos(t_q)|0> + sin(t_q)|1>
    th = rng.uniform(0.15, 1.4, size=n)
    f = torch.tensor(np.stack([np.cos(th), np.sin(th)], axis=1), dtype=torch.float64, device="cuda")
    v = torch.ones(1, dtype=torch.float64, device="cuda")
    for q in range(n - 1, -1, -1):   # qubit n-1 is the most significant factor
        v = (v[:, None] * f[q][None, :]).reshape(-1)
    st = torch.complex(v.float(), torch.zeros_like(v, dtype=torch.float32))
    del v
    torch.cuda.empty_cache()
    c2, s2 = np.cos(th) ** 2, np.sin(th) ** 2
    for r in range(1, n + 1):
        qs = _qubit_orders(n, r, rng)[r % 3]
        p = qsv.qsv_probabilities(st, qs)
        ms = rng.integers(1 << r, size=64)
        got = p[torch.from_numpy(ms).cuda()].cpu().numpy()
        want = np.array([np.prod([s2[q] if b else c2[q] for q, b in zip(qs, _outcome_bits(int(m), qs))]) for m in ms])
        # each stored amplitude carries one complex64 rounding of the exact
        # product, so each |psi_i|^2 and every outcome sum is within 2^-23
        # relative of the closed form
        assert np.all(np.abs(got - want) <= 1e-6 * want), (r, qs)
        assert abs(float(p.sum().item()) - 1.0) <= 1e-6, r
        del p


def test_sampled_outcomes_random_state_30q(gpu):
    """Brute force over the stored amplitudes: for r >= 14 each outcome sums
    at most 2^16 amplitudes, gathered on the host by their indices."""
    import torch
    n = 30
    g = torch.Generator(device="cuda").manual_seed(5)
    st = torch.randn(1 << n, dtype=torch.complex64, device="cuda", generator=g)
    host = st.cpu().numpy()
    rng = np.random.default_rng(11)
    for r in range(14, n + 1):
        qs = _qubit_orders(n, r, rng)[r % 3]
        p = qsv.qsv_probabilities(st, qs)
        others = [q for q in range(n) if q not in qs]
        rest = np.arange(1 << (n - r), dtype=np.int64)
        base_rest = np.zeros_like(rest)
        for k, q in enumerate(others):
            base_rest |= ((rest >> k) & 1) << q
        for m in rng.integers(1 << r, size=4):
            idx = base_rest.copy()
            for q, b in zip(qs, _outcome_bits(int(m), qs)):
                idx |= b << q
            amp = host[idx].astype(np.complex128)
            want = float(np.sum(amp.real ** 2 + amp.imag ** 2))
            got = float(p[int(m)].item())
            # 2^(n-r) non-negative terms summed in two orders
            assert abs(got - want) <= 2.0 ** (n - r + 1 - 53) * want, (r, qs, int(m))
        del p


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_swap_only_pass_is_exact(gpu, dt, seed):
    """A pass whose gates are SWAPs of local qubits only relabels positions:
    threads store where other threads loaded, so every load of the tile must
    complete before the first store.  The result is the oracle's permutation,
    bit for bit."""
    import torch
    n = 16
    local = list(range(12)) if dt == qsv.QSV_C64 else list(range(11))
    rng = np.random.default_rng(seed)
    circ = []
    for _ in range(6 + 3 * seed):
        a, b = [int(x) for x in rng.choice(local, 2, replace=False)]
        circ.append(W.gate("SWAP", [a, b]))
    psi0 = W.random_state(n, seed)
    if dt == qsv.QSV_C64:
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    t = torch.complex64 if dt == qsv.QSV_C64 else torch.complex128
    st = torch.from_numpy(psi0).to(t).cuda()
    qsv.qsv_run_pass(st, circ, local)
    assert np.array_equal(st.cpu().numpy().astype(np.complex128), S.run_circuit(psi0, circ))
