"""Learned cost model for plan selection: record, train, save, load.

Timings are recorded by the simulator itself: candidate plans (per-gate,
greedy fusion kmax 2..5, LDS passes) are built for synthetic circuits and
every op is timed alone with HIP events; each sample is the op's feature
vector (``qsv_plan_op_features``) and the log of its median run time.  Two
sources of samples: random fused blocks (Haar-random k-qubit unitaries,
k = 2..6, on 26..33 qubits, targets low, high or mixed), each timed as a
dense VALU gate and, for k >= 4, as a matrix-core block; and the ops of the
candidate plans of synthetic circuits (QFT, supremacy-like, variational,
random).  The MLP (13 -> 64 -> 64 -> 1, ReLU) is trained on the GPU with the
library's own forward / backward / Adam kernels.  ``load_into_library`` hands the
weights to ``qsv_cost_model_set`` so that ``PLAN_LEARNED`` can score plans.

Usage (on a GPU):  python -m paper_2203_08826_amd.cost_model --out model.npz
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import (COST_FEATURES, PLAN_GREEDY, PLAN_PASSES, PLAN_PER_GATE, QSV_C64, QSV_C128, qsv_cost_model_set,
               qsv_mlp_adam, qsv_mlp_backward, qsv_mlp_forward, qsv_mlp_param_count, qsv_plan_create,
               qsv_plan_execute_ops, qsv_plan_op_features, qsv_plan_stats_get)

SIZES = [COST_FEATURES, 64, 64, 1]
DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_model.npz")


def candidate_configs(n, dtype, jit=(0, 1)):
    """The plans the learned planner chooses among (mirrors build_learned),
    with the LDS passes interpreted and compiled."""
    out = [("per_gate", dict(mode=PLAN_PER_GATE))]
    for k in range(2, 6):
        out.append(("greedy%d" % k, dict(mode=PLAN_GREEDY, kmax=k, use_mfma=1)))
    for j in jit:
        ld = (5 if dtype == QSV_C64 else 4) + (9 if j else 8)   # compiled passes: 512-thread workgroups
        sfx = "_jit" if j else ""
        if n >= ld:
            out.append(("passes%d%s" % (ld, sfx), dict(mode=PLAN_PASSES, local_bits=ld, jit=j)))
        if n >= ld - 1:
            out.append(("passes%d%s" % (ld - 1, sfx), dict(mode=PLAN_PASSES, local_bits=ld - 1, jit=j)))
    return out


def time_ops(plan, state, nops, reps=3, max_ops=None, rng=None):
    """(features, median seconds) of ops of a plan, each run alone."""
    import torch
    idx = list(range(nops))
    if max_ops is not None and nops > max_ops:
        idx = sorted(rng.choice(nops, size=max_ops, replace=False).tolist())
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    feats, secs = [], []
    for i in idx:
        qsv_plan_execute_ops(plan, state, i, 1)   # warm
        ts = []
        for _ in range(reps):
            e0.record(s)
            qsv_plan_execute_ops(plan, state, i, 1)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        feats.append(qsv_plan_op_features(plan, i))
        secs.append(float(np.median(ts)))
    return np.array(feats, dtype=np.float32), np.array(secs)


def plan_time(plan, state, nops):
    """Measured seconds of a whole plan (sum of per-op medians is not used)."""
    import torch
    torch.cuda.synchronize()
    from . import qsv_plan_execute
    qsv_plan_execute(plan, state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qsv_plan_execute(plan, state)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def record(circuits, dtypes=(QSV_C64,), max_ops=24, seed=0, log=None):
    """circuits: list of (name, n, gate list).  Returns features X, log-seconds y, meta."""
    import torch
    rng = np.random.default_rng(seed)
    X, y, meta = [], [], []
    for name, n, circ in circuits:
        for dt in dtypes:
            tdt = torch.complex64 if dt == QSV_C64 else torch.complex128
            st = torch.randn(1 << n, dtype=tdt, device="cuda")
            st /= torch.linalg.vector_norm(st)
            for cname, kw in candidate_configs(n, dt):
                plan = qsv_plan_create(n, dt, circ, **kw)
                nops = qsv_plan_stats_get(plan)["n_launches"]
                f, s = time_ops(plan, st, nops, max_ops=max_ops, rng=rng)
                X.append(f)
                y.append(np.log(s))
                meta += [(name, n, dt, cname)] * len(s)
                if log:
                    log("recorded %s n=%d dt=%d %s: %d ops, median %.3f ms" % (name, n, dt, cname, len(s),
                                                                           1e3 * float(np.median(s))))
            del st
            torch.cuda.empty_cache()
    return np.concatenate(X), np.concatenate(y).astype(np.float32), meta


def random_blocks(count, ns=range(26, 34), ks=range(2, 7), seed=0):
    """Random fused blocks: (n, targets, unitary) with n and k uniform, the
    targets drawn among the lowest 8 qubits, the highest 8, or anywhere (a
    third each), Haar-random unitaries (QR of complex Gaussians)."""
    import workloads as W
    rng = np.random.default_rng(seed)
    ns, ks = list(ns), list(ks)
    out = []
    for _ in range(count):
        n = int(rng.choice(ns))
        k = int(rng.choice(ks))
        mode = int(rng.integers(3))
        pool = list(range(8)) if mode == 0 else list(range(n - 8, n)) if mode == 1 else list(range(n))
        tg = [int(q) for q in rng.choice(pool, size=k, replace=False)]
        out.append((n, tg, W.random_unitary(k, rng)))
    return out


def record_blocks(blocks, reps=5, log=None):
    """Each block timed alone (median of `reps` after one warm-up) as a dense
    gate, and for k >= 4 on complex64 as a matrix-core block."""
    import torch
    import workloads as W
    X, y = [], []
    by_n = {}
    for b in blocks:
        by_n.setdefault(b[0], []).append(b)
    for n in sorted(by_n):
        st = torch.randn(1 << n, dtype=torch.complex64, device="cuda")
        st /= torch.linalg.vector_norm(st)
        for _, tg, u in by_n[n]:
            g = W.gate("UNITARY", tg)
            g["matrix"] = u
            kinds = [dict(mode=PLAN_PER_GATE)]
            if len(tg) >= 4:
                kinds.append(dict(mode=PLAN_GREEDY, kmax=len(tg), use_mfma=1))
            for kw in kinds:
                plan = qsv_plan_create(n, QSV_C64, [g], **kw)
                f, sec = time_ops(plan, st, qsv_plan_stats_get(plan)["n_launches"], reps=reps)
                X.append(f)
                y.append(np.log(sec))
        if log:
            log("recorded %d blocks at n=%d" % (len(by_n[n]), n))
        del st
        torch.cuda.empty_cache()
    return np.concatenate(X), np.concatenate(y).astype(np.float32)


def init_params(rng, sizes=SIZES):
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((a, b)) * math.sqrt(2.0 / a)).reshape(-1))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def normalisation(X):
    mean = X.mean(axis=0)
    scale = X.std(axis=0)
    scale[scale < 1e-6] = 1.0
    return mean.astype(np.float32), scale.astype(np.float32)


def train(X, y, steps=3000, lr=3e-3, seed=0, log=None):
    """Full-batch Adam on the GPU kernels; returns (params, mean, scale, final mse)."""
    import torch
    rng = np.random.default_rng(seed)
    mean, scale = normalisation(X)
    Xn = ((X - mean) / scale).astype(np.float32)
    B = Xn.shape[0]
    p = torch.from_numpy(init_params(rng)).cuda()
    assert p.numel() == qsv_mlp_param_count(SIZES)
    dX = torch.from_numpy(Xn).cuda()
    dy = torch.from_numpy(y.astype(np.float32)).cuda()
    acts = torch.empty(B * sum(SIZES[1:]), dtype=torch.float32, device="cuda")
    pred = torch.empty(B, dtype=torch.float32, device="cuda")
    g = torch.empty_like(p)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    scratch = torch.empty(2 * B * max(SIZES), dtype=torch.float32, device="cuda")
    for step in range(1, steps + 1):
        qsv_mlp_forward(p, SIZES, dX, acts, pred)
        qsv_mlp_backward(p, SIZES, dX, acts, pred, dy, g, scratch)
        qsv_mlp_adam(p, g, m, v, step, lr=lr)
        if log and (step % 500 == 0 or step == 1):
            log("step %d mse %.4f" % (step, float(((pred - dy) ** 2).mean())))
    qsv_mlp_forward(p, SIZES, dX, acts, pred)
    mse = float(((pred - dy) ** 2).mean())
    return p.cpu().numpy(), mean, scale, mse


def predict(params, mean, scale, X):
    import torch
    Xn = torch.from_numpy(((X - mean) / scale).astype(np.float32)).cuda()
    B = Xn.shape[0]
    acts = torch.empty(B * sum(SIZES[1:]), dtype=torch.float32, device="cuda")
    pred = torch.empty(B, dtype=torch.float32, device="cuda")
    qsv_mlp_forward(torch.from_numpy(params).cuda(), SIZES, Xn, acts, pred)
    return pred.cpu().numpy()


def save(path, params, mean, scale, info=None):
    np.savez(path, params=params, sizes=np.array(SIZES, dtype=np.int32), mean=mean, scale=scale,
             info=np.array(json.dumps(info or {})))


def load(path):
    d = np.load(path, allow_pickle=False)
    return d["params"], [int(s) for s in d["sizes"]], d["mean"], d["scale"]


def load_into_library(path=DEFAULT_PATH):
    params, sizes, mean, scale = load(path)
    qsv_cost_model_set(params, sizes, mean, scale)


def training_circuits(ns=(24, 26, 28, 30), seed=0):
    import workloads as W
    out = []
    for n in ns:
        out.append(("qft", n, W.qft(n)))
        out.append(("supremacy", n, W.supremacy(n, 8, seed=seed + n)))
        out.append(("variational", n, W.variational(n, 4, seed=seed + n)))
        out.append(("random", n, W.random_circuit(n, 60, seed=seed + n, kmax=3, max_controls=1)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--ns", default="26,28,30,32")
    ap.add_argument("--blocks", type=int, default=600, help="random fused blocks (k = 2..6, n = 26..33)")
    ap.add_argument("--max-ops", type=int, default=24)
    ap.add_argument("--steps", type=int, default=3000)
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    ns = tuple(int(x) for x in args.ns.split(","))
    t0 = time.perf_counter()
    Xb, yb = record_blocks(random_blocks(args.blocks), log=log)
    log("recorded %d block samples in %.1f s" % (len(yb), time.perf_counter() - t0))
    X, y, meta = record(training_circuits(ns), dtypes=(QSV_C64, QSV_C128), max_ops=args.max_ops, log=log)
    log("recorded %d plan-op samples in %.1f s" % (len(y), time.perf_counter() - t0))
    X = np.concatenate([Xb, X])
    y = np.concatenate([yb, y])
    # hold out 20% (by sample, seeded) for the prediction-error report
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(y))
    cut = int(0.8 * len(y))
    tr, te = perm[:cut], perm[cut:]
    params, mean, scale, mse = train(X[tr], y[tr], steps=args.steps, log=log)
    pte = predict(params, mean, scale, X[te])
    err = float(np.median(np.abs(np.exp(pte - y[te]) - 1.0)))
    info = {"samples": int(len(y)), "block_samples": int(len(yb)), "train_mse_log": mse,
            "heldout_median_rel_err": err, "ns": list(ns)}
    log("train mse(log s) %.4f, held-out median relative error %.3f" % (mse, err))
    # final model on all samples
    params, mean, scale, mse = train(X, y, steps=args.steps)
    save(args.out, params, mean, scale, info)
    np.savez(os.path.splitext(args.out)[0] + "_data.npz", X=X, y=y)
    log(json.dumps(info))


if __name__ == "__main__":
    sys.exit(main())
