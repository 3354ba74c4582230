"""GPU parity of the measurement operators (methodology section, Sec. 2):
collapse and re-normalisation, inverse-CDF shot sampling and Metropolis shot
frequencies, against the oracle, through the C ABI.  Random numbers are
seeded inputs shared by both sides."""
import math

import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import measure as OM
from oracle import statevec as S

pytestmark = pytest.mark.gpu


def _dev(psi, dt):
    import torch
    t = torch.complex64 if dt == "c64" else torch.complex128
    return torch.from_numpy(np.asarray(psi, dtype=np.complex128)).to(t).cuda().contiguous()


def _as_stored(psi, dt):
    return np.asarray(psi, dtype=np.complex64 if dt == "c64" else np.complex128).astype(np.complex128)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 5, 12, 17])
def test_collapse_matches_oracle(gpu, dt, n):
    rng = np.random.default_rng(20 + n)
    psi = _as_stored(W.random_state(n, 9), dt)
    for r in sorted({1, min(3, n), n}):
        qs = [int(q) for q in rng.permutation(n)[:r]]
        for m in sorted({0, (1 << r) - 1, int(rng.integers(1 << r))}):
            st = _dev(psi, dt)
            p = float(qsv.qsv_collapse(st, qs, m).cpu().numpy()[0])
            want, pw = OM.collapse(psi, qs, m)
            # p: 2^(n-r) non-negative float64 terms summed in two orders
            assert abs(p - pw) <= 2.0 ** (n - r + 1 - 53) * pw + 1e-300, (r, qs, m)
            got = st.cpu().numpy().astype(np.complex128)
            # complex64: the kept amplitudes are rounded once more after the
            # float64 scaling (relative 2^-24); complex128 within 1e-12
            tol = 2.0 ** -23 * np.max(np.abs(want)) if dt == "c64" else 1e-12
            assert np.max(np.abs(got - want)) <= tol, (r, qs, m)
            # every amplitude outside the outcome is exactly 0
            assert not np.any(got[~OM.projector_mask(n, qs, m)])


def test_collapse_impossible_outcome_zeroes_the_state(gpu):
    n = 6
    st = _dev(S.basis_state(n, 0b101101), "c128")
    p = float(qsv.qsv_collapse(st, [0], 0).cpu().numpy()[0])
    assert p == 0.0 and not st.abs().max().item()


def test_collapse_30q_closed_forms(gpu):
    """GHZ: measuring qubit 17 as 1 leaves |1..1> exactly (1/sqrt(p) times a
    stored amplitude a with p = 2 a^2... re-normalised to 1 within one
    rounding).  Product state: collapsing qubits (3, 20, 29) leaves the product
    of the other qubits' factors."""
    import torch
    n = 30
    N = 1 << n
    st = torch.zeros(N, dtype=torch.complex64, device="cuda")
    a = np.float32(1 / math.sqrt(2))
    st[0] = complex(a)
    st[N - 1] = complex(a)
    p = float(qsv.qsv_collapse(st, [17], 1).cpu().numpy()[0])
    assert p == float(a) * float(a)
    assert int(torch.count_nonzero(st).item()) == 1
    assert abs(complex(st[N - 1].item()) - 1.0) <= 2.0 ** -23
    del st
    torch.cuda.empty_cache()
    rng = np.random.default_rng(4)
    th = rng.uniform(0.15, 1.4, size=n)
    f = torch.tensor(np.stack([np.cos(th), np.sin(th)], axis=1), dtype=torch.float64, device="cuda")
    v = torch.ones(1, dtype=torch.float64, device="cuda")
    for q in range(n - 1, -1, -1):
        v = (v[:, None] * f[q][None, :]).reshape(-1)
    st = torch.complex(v.float(), torch.zeros_like(v, dtype=torch.float32))
    del v
    torch.cuda.empty_cache()
    qs, m = [3, 20, 29], 0b101   # qubit 3 -> 1, 20 -> 0, 29 -> 1
    p = float(qsv.qsv_collapse(st, qs, m).cpu().numpy()[0])
    pw = np.sin(th[3]) ** 2 * np.cos(th[20]) ** 2 * np.sin(th[29]) ** 2
    assert abs(p - pw) <= 1e-6 * pw
    # sampled kept amplitudes: product of the unmeasured factors
    idx = rng.integers(N, size=4096)
    idx = (idx | (1 << 3) | (1 << 29)) & ~(1 << 20)
    got = st[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    want = np.ones(idx.size)
    for q in range(n):
        if q in qs:
            continue
        want *= np.where((idx >> q) & 1, np.sin(th[q]), np.cos(th[q]))
    assert np.max(np.abs(got - want) / np.abs(want)) <= 2e-6
    assert abs(float(qsv.qsv_norm2(st).cpu().numpy()[0]) - 1.0) <= 1e-6


def _probs(r, seed):
    """A seeded probability vector over 2^r outcomes with a few zeros."""
    rng = np.random.default_rng(seed)
    p = rng.random(1 << r) ** 4
    p[rng.integers(1 << r, size=max(1, (1 << r) // 16))] = 0.0
    return p / p.sum()


@pytest.mark.parametrize("r", [1, 4, 10, 12, 17])
def test_inverse_cdf_matches_oracle(gpu, r):
    import torch
    rng = np.random.default_rng(100 + r)
    p = _probs(r, r)
    u = rng.random(50000)
    u[:3] = [0.0, 0.5, 1.0 - 2.0 ** -53]
    dp = torch.from_numpy(p).cuda()
    cdf, sm, ct = qsv.qsv_sample_cdf(dp, torch.from_numpy(u).cuda())
    c_or = OM.cumulative(p)
    # 2^r non-negative terms summed in two orders
    assert np.max(np.abs(cdf.cpu().numpy() - c_or)) <= 2.0 ** (r + 1 - 53)
    got = sm.cpu().numpy()
    want = OM.sample_inverse_cdf(p, u)
    diff = np.nonzero(got != want)[0]
    # a draw may differ only where u T lies within rounding of a boundary c_m
    x = u * c_or[-1]
    for s in diff:
        b = c_or[min(got[s], want[s])]
        assert abs(x[s] - b) <= 2.0 ** (r + 2 - 53), (s, got[s], want[s])
    assert diff.size <= 2
    assert np.array_equal(ct.cpu().numpy().astype(np.int64), np.bincount(got, minlength=1 << r))
    assert not np.any(p[got] == 0.0)


def test_inverse_cdf_chi_square_20_bits(gpu):
    import torch
    from scipy import stats
    r = 20
    p = _probs(r, 7)
    N = 1 << 22
    u = torch.rand(N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    _, _, ct = qsv.qsv_sample_cdf(torch.from_numpy(p).cuda(), u, samples=False)
    counts = ct.cpu().numpy().astype(np.float64)
    assert counts.sum() == N
    # pool the outcomes into 256 bins of consecutive outcomes for the test
    pb = p.reshape(256, -1).sum(axis=1)
    cb = counts.reshape(256, -1).sum(axis=1)
    chi2 = float(np.sum((cb - N * pb) ** 2 / (N * pb)))
    assert chi2 <= stats.chi2.ppf(0.9999, 255)


@pytest.mark.parametrize("r,C,T", [(1, 3, 50), (5, 64, 200), (12, 1000, 64), (16, 4096, 16)])
def test_metropolis_matches_oracle(gpu, r, C, T):
    """Same probabilities, starts, proposals and uniforms on both sides: the
    acceptance test u p(x) < p(y) is one float64 product and comparison, so
    the frequencies agree exactly."""
    import torch
    rng = np.random.default_rng(200 + r)
    p = _probs(r, 50 + r)
    starts = rng.integers(1 << r, size=C)
    prop = rng.integers(1 << r, size=(T, C))
    uni = rng.random((T, C))
    got = qsv.qsv_sample_metropolis(torch.from_numpy(p).cuda(), torch.from_numpy(starts).cuda(),
                                    torch.from_numpy(prop).cuda(), torch.from_numpy(uni).cuda())
    want = OM.metropolis_counts(p, starts, prop, uni)
    assert np.array_equal(got.cpu().numpy().astype(np.int64), want)


def test_sampling_from_measured_state(gpu):
    """Probabilities of a circuit's state feed both samplers: frequencies
    converge to the probabilities."""
    import torch
    n, qs = 14, [13, 2, 7, 0, 9]
    st = _dev(S.run_circuit(S.basis_state(n, 0), W.supremacy(n, 6, seed=2)), "c128")
    p = qsv.qsv_probabilities(st, qs)
    N = 1 << 20
    u = torch.rand(N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    _, _, ct = qsv.qsv_sample_cdf(p, u, samples=False)
    pw = p.cpu().numpy()
    assert np.max(np.abs(ct.cpu().numpy() / N - pw)) <= 5.0 * math.sqrt(0.25 / N)
    g = torch.Generator("cuda").manual_seed(2)
    C, T = 2048, 512
    starts = torch.randint(0, 32, (C,), device="cuda", generator=g)
    prop = torch.randint(0, 32, (T, C), device="cuda", generator=g)
    uni = torch.rand((T, C), dtype=torch.float64, device="cuda", generator=g)
    counts = qsv.qsv_sample_metropolis(p, starts, prop, uni).cpu().numpy().astype(np.float64)
    assert counts.sum() == C * T
    assert np.max(np.abs(counts / (C * T) - pw)) <= 0.01
