"""GPU MLP kernels (cost model) against the oracle's float64 numpy MLP."""
import math

import numpy as np
import pytest

import paper_2203_08826_amd as qsv
from oracle import mlp as OM

pytestmark = pytest.mark.gpu

SIZES = [12, 32, 16, 1]


def _init(rng, sizes):
    params = [(rng.standard_normal((a, b)) / math.sqrt(a), 0.1 * rng.standard_normal(b))
              for a, b in zip(sizes[:-1], sizes[1:])]
    flat = np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)
    return params, flat


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _unflat(flat, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, flat[o:o + b]))
        o += b
    return out


# the shipped cost model's network (13 features -> 64 -> 64 -> 1) at the
# batch of its training set, besides a small network at small batches
SHIPPED = [qsv.COST_FEATURES, 64, 64, 1]


@pytest.mark.parametrize("sizes,batch", [(SIZES, 1), (SIZES, 7), (SIZES, 300), (SHIPPED, 4800)])
def test_forward_backward_match_oracle(gpu, sizes, batch):
    import torch
    SIZES = sizes
    rng = np.random.default_rng(batch)
    params, flat = _init(rng, SIZES)
    params = _unflat(flat.astype(np.float64), SIZES)   # the GPU's float32 values, in float64
    X = rng.standard_normal((batch, SIZES[0])).astype(np.float32)
    t = rng.standard_normal(batch).astype(np.float32)
    assert qsv.qsv_mlp_param_count(SIZES) == flat.size
    dp, dX, dt = _dev(flat), _dev(X), _dev(t)
    acts = torch.empty(batch * sum(SIZES[1:]), dtype=torch.float32, device="cuda")
    pred = torch.empty(batch, dtype=torch.float32, device="cuda")
    qsv.qsv_mlp_forward(dp, SIZES, dX, acts, pred)
    want, cache = OM.forward(params, X.astype(np.float64))
    got = pred.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-4 * (1 + np.max(np.abs(want)))
    grads = torch.empty_like(dp)
    scratch = torch.empty(2 * batch * max(SIZES), dtype=torch.float32, device="cuda")
    qsv.qsv_mlp_backward(dp, SIZES, dX, acts, pred, dt, grads, scratch)
    gw = OM.backward(params, cache, want, t.astype(np.float64))
    gflat = np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in gw])
    g = grads.cpu().numpy()
    assert np.max(np.abs(g - gflat)) <= 1e-4 * (1 + np.max(np.abs(gflat)))


def test_adam_matches_oracle(gpu):
    rng = np.random.default_rng(0)
    p = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros(1000, np.float32)
    v = np.zeros(1000, np.float32)
    dp, dm, dv = _dev(p), _dev(m), _dev(v)
    pp, mm, vv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 6):
        g = rng.standard_normal(1000).astype(np.float32)
        qsv.qsv_mlp_adam(dp, _dev(g), dm, dv, step, lr=1e-2)
        pp, mm, vv = OM.adam_step(pp, g.astype(np.float64), mm, vv, step, lr=1e-2)
    assert np.max(np.abs(dp.cpu().numpy() - pp)) <= 1e-5


def test_training_reduces_loss(gpu):
    """A few hundred Adam steps of the GPU kernels fit a smooth target."""
    import torch
    rng = np.random.default_rng(1)
    _, flat = _init(rng, SIZES)
    X = rng.standard_normal((256, SIZES[0])).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    dp, dX, dt = _dev(flat), _dev(X), _dev(t)
    acts = torch.empty(256 * sum(SIZES[1:]), dtype=torch.float32, device="cuda")
    pred = torch.empty(256, dtype=torch.float32, device="cuda")
    grads = torch.empty_like(dp)
    m = torch.zeros_like(dp)
    v = torch.zeros_like(dp)
    scratch = torch.empty(2 * 256 * max(SIZES), dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 401):
        qsv.qsv_mlp_forward(dp, SIZES, dX, acts, pred)
        if step in (1, 400):
            losses.append(float(((pred - dt) ** 2).mean()))
        qsv.qsv_mlp_backward(dp, SIZES, dX, acts, pred, dt, grads, scratch)
        qsv.qsv_mlp_adam(dp, grads, m, v, step, lr=3e-3)
    assert losses[1] < 0.2 * losses[0]
