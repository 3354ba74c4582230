"""GPU parity of the float64 reductions against the oracle."""
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
    # the oracle sees exactly the amplitudes the GPU holds
    return np.asarray(psi, dtype=np.complex64 if dt == "c64" else np.complex128).astype(np.complex128)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 5, 14, 18])
def test_norm_inner(gpu, dt, n):
    a = _as_stored(W.random_state(n, 1), dt)
    b = _as_stored(W.random_state(n, 2), dt)
    da, db = _dev(a, dt), _dev(b, dt)
    nrm = qsv.qsv_norm2(da).cpu().numpy()[0]
    assert abs(nrm - S.norm2(a)) <= 1e-13
    ip = qsv.qsv_inner(da, db).cpu().numpy()
    want = S.inner(a, b)
    assert abs(ip[0] - want.real) <= 1e-13 and abs(ip[1] - want.imag) <= 1e-13
    # reproducible bit for bit
    assert qsv.qsv_norm2(da).cpu().numpy()[0] == nrm


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [4, 12, 17])
def test_probabilities(gpu, dt, n):
    rng = np.random.default_rng(n)
    psi = _as_stored(W.random_state(n, 3), dt)
    d = _dev(psi, dt)
    for r in sorted({1, 2, min(n, 5), n - 1, n} - {0}):
        qs = [int(q) for q in rng.permutation(n)[:r]]
        got = qsv.qsv_probabilities(d, qs).cpu().numpy()
        want = S.probabilities(psi, qs)
        # 2^(n-r) non-negative float64 terms summed in two orders
        assert np.max(np.abs(got - want)) <= 2.0 ** (n - r + 1 - 53) + 1e-16, (r, qs)
        assert abs(got.sum() - S.norm2(psi)) <= 1e-12


def test_probabilities_ghz(gpu):
    n = 12
    st = _dev(S.run_circuit(S.basis_state(n, 0), W.ghz(n)), "c64")
    p = qsv.qsv_probabilities(st, [11, 0]).cpu().numpy()
    assert np.allclose(p, [0.5, 0, 0, 0.5], atol=1e-7)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [2, 3, 9, 12, 13, 15, 18, 19, 21, 23])
@pytest.mark.parametrize("periodic", [False, True])
def test_tfim_energy_and_apply(gpu, dt, n, periodic):
    """The energy's and H psi's sweeps (bits 0..11 first; then bits 0..5
    with 7 new bits per sweep for complex64, 6 for complex128) at sizes with
    one sweep (2, 3, 9, 12), with a last sweep that carries bits an earlier
    sweep summed (13, 15, 21, 23; 19 for complex128) and with only full later
    sweeps (19 for complex64, 18 for complex128)."""
    import torch
    psi = _as_stored(W.random_state(n, 4), dt)
    d = _dev(psi, dt)
    e = qsv.qsv_expval_zz_x(d, 1.0, 0.5, periodic).cpu().numpy()[0]
    assert abs(e - S.expval_tfim(psi, 1.0, 0.5, periodic)) <= 1e-12
    out = torch.empty_like(d)
    qsv.qsv_apply_tfim(d, out, 1.0, 0.5, periodic)
    want = S.apply_h_tfim(psi, 1.0, 0.5, periodic)
    tol = 1e-5 * n if dt == "c64" else 1e-12
    assert np.max(np.abs(out.cpu().numpy() - want)) <= tol


def test_product_state_energies(gpu):
    n = 10
    zero = _dev(S.basis_state(n, 0), "c128")
    assert abs(qsv.qsv_expval_zz_x(zero, 1.0, 0.5).cpu().numpy()[0] - (n - 1)) <= 1e-13
    plus = _dev(np.full(1 << n, 2 ** (-n / 2), complex), "c128")
    assert abs(qsv.qsv_expval_zz_x(plus, 1.0, 0.5).cpu().numpy()[0] - 0.5 * n) <= 1e-12
