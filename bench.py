"""Benchmark: 30-qubit QFT, complex64, on one MI355X.

A step is one application of the whole QFT circuit (n H gates, n(n-1)/2
controlled phases, n/2 SWAPs) to a 2^n complex64 state resident in HBM,
with the plan the library picks (LDS passes scored by the cost model when
one is loaded; passes compiled into kernels of their own unless --jit 0).
Also reported: the same circuit as plain per-gate complex128, per-gate /
greedy-fused complex64 and interpreted LDS passes, the complex64 state's
infidelity against the complex128 one, a closed-form check of sampled
amplitudes, the roofline of the dominant kernel and the oracle timed on the
host cores.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFLOPS = 157.3   # dense FP32 MFMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--plan", default="learned", choices=["per_gate", "greedy", "passes", "learned"])
    ap.add_argument("--kmax", type=int, default=2)
    ap.add_argument("--jit", type=int, default=1, choices=[0, 1], help="compile the LDS passes (1) or interpret them (0)")
    ap.add_argument("--no-baselines", action="store_true", help="skip the per-gate / c128 comparison plans")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle sample: the first gates of the circuit, until this many seconds have run")
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2203_08826_amd", "cost_model.npz"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain device copy of 2^n complex64 (counter calibration)")
    ap.add_argument("--stream-calibration", action="store_true",
                    help="only time the in-place stream (qsv_scale) and torch's copy: the measured ceilings")
    ap.add_argument("--workload", default="qft", choices=["qft", "supremacy", "variational", "adjoint", "learned", "single_gate", "qft20",
                             "cpu_baseline_full", "adiabatic", "sliced", "reductions"],
                    help="qft: the headline line; the others print their own configuration's line")
    ap.add_argument("--depth", type=int, default=20)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--time", type=float, default=2.0, help="adiabatic: total time T")
    ap.add_argument("--dt", type=float, default=0.05, help="adiabatic: Trotter step")
    return ap.parse_args()


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _zero_state(n, dtype):
    import torch
    st = torch.zeros(1 << n, dtype=dtype, device="cuda")
    st[0] = 1.0
    return st


def _infidelity(qsv, a, b):
    """1 - |<a|b>|^2 / (<a|a><b|b>), float64 sums (the states are widened only
    when their dtypes differ)."""
    import torch
    if a.dtype != b.dtype:
        a = a.to(torch.complex128)
        b = b.to(torch.complex128)
    ov = qsv.qsv_inner(a, b).cpu().numpy()
    na = qsv.qsv_norm2(a).cpu().numpy()[0]
    nb = qsv.qsv_norm2(b).cpu().numpy()[0]
    return float(1.0 - (ov[0] ** 2 + ov[1] ** 2) / (na * nb))


def workload_supremacy(args):
    """Random supremacy-like circuit: per-gate kernels vs LDS passes, c64 and c128."""
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    n = args.n
    circ = W.supremacy(n, args.depth, seed=0)
    out = {"metric": "circuit s & HBM GB/s", "config": {"workload": "supremacy-like n=%d depth=%d (%d gates)" % (
        n, args.depth, len(circ))}, "results": {}}
    for dname, dt, tdt in (("c64", qsv.QSV_C64, torch.complex64), ("c128", qsv.QSV_C128, torch.complex128)):
        for pname, mode, jit in (("per_gate", qsv.PLAN_PER_GATE, 0), ("passes", qsv.PLAN_PASSES, 0),
                                 ("passes_compiled", qsv.PLAN_PASSES, 1)):
            plan = qsv.qsv_plan_create(n, dt, circ, mode=mode, jit=jit)
            st = _zero_state(n, tdt)
            s = _timed(lambda: qsv.qsv_plan_execute(plan, st), 1)
            b = plan.stats()["bytes"]
            out["results"]["%s_%s" % (pname, dname)] = {"s": round(s, 4), "GB/s": round(b / s / 1e9, 1),
                                                        "launches": plan.stats()["n_launches"]}
            del st
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


_T0 = time.perf_counter()


def _progress(msg):
    """A progress line on stderr (long workloads print one per stage)."""
    print("[%7.1f s] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def workload_variational(args):
    """Variational ansatz fused into dense 5-qubit blocks on FP32 MFMA (c64),
    against the c128 reference (LDS passes, oracle-checked at small n)."""
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    n = args.n
    circ = W.variational(n, args.layers, seed=0)
    _progress("variational n=%d layers=%d: planning greedy kmax=5" % (n, args.layers))
    fused = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_GREEDY, kmax=5, use_mfma=1)
    fs = fused.stats()
    # flops the matrix cores execute: 8 * 2^k per amplitude for k = 4 (real
    # 2D x 2D form), 6 * 2^k for k = 5, 6 (three real D x D products)
    mfma_flops = 0.0
    for i in range(fs["n_launches"]):
        info = qsv.qsv_plan_op_info(fused, i)
        if info["kind"] == 1:
            k = int(round(math.log2(info["flops"] / (8.0 * 2.0 ** n))))
            mfma_flops += info["flops"] * (0.75 if k >= 5 else 1.0)
    a = _zero_state(n, torch.complex64)
    qsv.qsv_plan_execute(fused, a)
    torch.cuda.synchronize()
    t_fused = _timed(lambda: qsv.qsv_plan_execute(fused, a), 1)
    a = _zero_state(n, torch.complex64)
    qsv.qsv_plan_execute(fused, a)
    _progress("fused c64 %.4f s; c128 reference" % t_fused)
    ref_plan = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES)
    b = _zero_state(n, torch.complex128)
    t0 = time.perf_counter()
    qsv.qsv_plan_execute(ref_plan, b)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    infid = _infidelity(qsv, b, a)
    # the same circuit as compiled LDS passes (c64), parametric kernels: a
    # second circuit of the same ansatz with new angles reuses them
    _progress("reference %.3f s; compiling parametric passes" % t_ref)
    t0 = time.perf_counter()
    cp = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, jit=2)
    t_cp_create = time.perf_counter() - t0
    t0 = time.perf_counter()
    qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, args.layers, seed=1), mode=qsv.PLAN_PASSES, jit=2)
    t_rebind = time.perf_counter() - t0
    c = _zero_state(n, torch.complex64)
    qsv.qsv_plan_execute(cp, c)
    torch.cuda.synchronize()
    infid_cp = _infidelity(qsv, b, c)
    t_cp = _timed(lambda: qsv.qsv_plan_execute(cp, c), 1)
    print(json.dumps({"metric": "circuit s, TFLOP/s, infidelity vs c128", "config": {
        "workload": "variational n=%d layers=%d (%d gates), greedy kmax=5 on FP32 MFMA" % (n, args.layers, len(circ))},
        "fused_c64_s": round(t_fused, 4), "blocks": fs["n_blocks"], "mfma_blocks": fs["n_mfma_blocks"],
        "launches": fs["n_launches"], "GB/s": round(fs["bytes"] / t_fused / 1e9, 1),
        "TFLOP/s": round(fs["flops"] / t_fused / 1e12, 2),
        "matrix_core_TFLOP/s": round(mfma_flops / t_fused / 1e12, 2),
        "matrix_core_frac_of_fp32_peak": round(mfma_flops / t_fused / 1e12 / FP32_MATRIX_PEAK_TFLOPS, 4),
        "reference_c128_passes_s": round(t_ref, 4),
        "infidelity_c64_vs_c128": infid,
        "passes_compiled_parametric_c64": {"s": round(t_cp, 4), "launches": cp.stats()["n_launches"],
                                           "plan_create_s": round(t_cp_create, 2),
                                           "plan_create_new_angles_s": round(t_rebind, 3),
                                           "infidelity_vs_c128": infid_cp}}), flush=True)


def workload_adjoint(args):
    """Adjoint-method gradient of <H> (24-qubit hardware-efficient ansatz)."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    from paper_2203_08826_amd.autograd import expval
    n = args.n
    circ = W.variational(n, args.layers, seed=0)
    theta = torch.tensor([g["params"][0] for g in circ if g["name"] in ("RY", "RZ")], dtype=torch.float64,
                         device="cuda", requires_grad=True)

    def fwd_bwd(dt):
        th = theta.detach().clone().requires_grad_(True)
        e = expval(th, circ, n, dtype=dt)
        e.backward()
        return float(e.detach()), th.grad.detach().cpu().numpy()

    fwd_bwd(qsv.QSV_C64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e64, g64 = fwd_bwd(qsv.QSV_C64)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    e128, g128 = fwd_bwd(qsv.QSV_C128)
    # parameter shift on a seeded subset, with complex128 forward runs on the GPU
    from paper_2203_08826_amd.autograd import bind
    rng = np.random.default_rng(0)
    sub = sorted(rng.choice(theta.numel(), size=4, replace=False).tolist())
    ps = []
    for p in sub:
        vals = []
        for sh in (np.pi / 2, -np.pi / 2):
            th = theta.detach().clone()
            th[p] += sh
            vals.append(float(expval(th, circ, n, dtype=qsv.QSV_C128)))
        ps.append(0.5 * (vals[0] - vals[1]))
    print(json.dumps({"metric": "forward+backward s, gradient error", "config": {
        "workload": "hardware-efficient ansatz n=%d layers=%d, %d params, H = sum ZZ + 0.5 sum X" % (
            n, args.layers, theta.numel())},
        "fwd_bwd_c64_s": round(t, 4), "energy_c64": e64, "energy_c128": e128,
        "max_abs_grad_diff_c64_vs_c128": float(np.max(np.abs(g64 - g128))),
        "param_shift_subset": sub, "max_abs_c128_adjoint_vs_param_shift": float(np.max(np.abs(g128[sub] - np.array(ps))))}),
        flush=True)


def workload_learned(args):
    """Learned plan choice vs greedy fusion, the fixed rule "always compiled
    LDS passes" and unfused, complex64."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    from paper_2203_08826_amd import cost_model
    loaded = os.path.exists(args.model)
    if loaded:
        cost_model.load_into_library(args.model)
    n = args.n
    res = {}
    # dense 3-qubit unitaries in 5-qubit windows: fusing pays, passes cannot take them
    windows = W.dense_windows(n, seed=3)
    for name, circ in (("qft", W.qft(n)), ("supremacy_d30", W.supremacy(n, 30, seed=1)), ("dense_windows", windows)):
        row = {}
        states = {}
        for pname, kw in (("learned", dict(mode=qsv.PLAN_LEARNED, kmax=2, jit=args.jit)),
                          ("greedy2", dict(mode=qsv.PLAN_GREEDY, kmax=2)),
                          ("passes_compiled", dict(mode=qsv.PLAN_PASSES, jit=args.jit)),
                          ("unfused", dict(mode=qsv.PLAN_PER_GATE))):
            t0 = time.perf_counter()
            plan = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, **kw)
            t_create = time.perf_counter() - t0
            st = _zero_state(n, torch.complex64)
            if name == "qft":
                st[0] = 0
                st[W.basis_index(n, 0)] = 1
            s = _timed(lambda: qsv.qsv_plan_execute(plan, st), 1)
            ps = plan.stats()
            row[pname] = {"s": round(s, 4), "mode_used": ps["mode_used"], "predicted_s": ps["predicted_s"],
                          "plan_create_s": round(t_create, 2)}
            if pname in ("learned", "unfused"):
                states[pname] = st
            else:
                del st
            torch.cuda.empty_cache()
        row["infidelity_learned_vs_unfused"] = _infidelity(qsv, states["unfused"], states["learned"])
        idx = torch.randint(0, 1 << n, (1 << 20,), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
        row["max_abs_diff_sampled_2^20"] = float(torch.max(torch.abs(states["unfused"][idx] - states["learned"][idx])).item())
        del states
        torch.cuda.empty_cache()
        res[name] = row
    print(json.dumps({"metric": "measured s: learned vs greedy vs unfused", "config": {
        "workload": "QFT, supremacy-like depth 30 and 32 dense 3-qubit unitaries in four 5-qubit windows at n=%d, complex64" % n,
        "model_loaded": loaded}, "results": res}),
        flush=True)


def _touched_fraction(bits, pred, line_bits=0):
    """Fraction of the state a gate reads and writes: of its amplitudes
    (line_bits = 0), or of its 128-byte lines (line_bits = log2 of the
    amplitudes per line), when it changes exactly the amplitudes whose values
    of `bits` satisfy `pred`."""
    import itertools
    inside = [i for i, b in enumerate(bits) if b < line_bits]
    hit = 0
    outs = list(itertools.product([0, 1], repeat=len(bits) - len(inside)))
    for o in outs:
        if line_bits:   # a line counts when any of its amplitudes is touched
            ok = False
            for v_in in itertools.product([0, 1], repeat=len(inside)):
                v, it_in, it_out = [], iter(v_in), iter(o)
                for i in range(len(bits)):
                    v.append(next(it_in) if i in inside else next(it_out))
                ok = ok or bool(pred(v))
            hit += ok
        else:
            hit += bool(pred(list(o)))
    return hit / len(outs)


def workload_reductions(args):
    """Measurement-side kernels at n qubits (complex64 and complex128, random
    state): probabilities of r measured qubits for several r and qubit sets,
    the norm, the TFIM energy and H psi, a collapse, and inverse-CDF sampling of 2^20
    shots from 2^20 outcomes; each timed with HIP events on the launch stream
    over --steps calls, GB/s of algorithmic bytes (state read, plus outputs)."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    n = args.n
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(0)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3 / args.steps

    res = {}
    for dname, tdt, s in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        g = torch.Generator(device="cuda").manual_seed(1)
        st = torch.randn(1 << n, dtype=tdt, device="cuda", generator=g)
        st /= torch.linalg.vector_norm(st)
        state_bytes = (1 << n) * s
        cases = []
        for r, label in ((1, "top"), (4, "low"), (10, "mixed"), (16, "mixed"), (20, "mixed"), (24, "mixed"), (n, "all")):
            if label == "top":
                qs = [n - 1]
            elif label == "low":
                qs = list(range(r))
            elif label == "all":
                qs = list(range(n - 1, -1, -1))
            else:
                qs = [int(q) for q in rng.choice(n, size=r, replace=False)]
            out = torch.empty(1 << r, dtype=torch.float64, device="cuda")
            cases.append(("probs_r%d_%s" % (r, label), lambda qs=qs, out=out: qsv.qsv_probabilities(st, qs, out=out),
                          state_bytes + (1 << r) * 8))
        nout = torch.empty(1, dtype=torch.float64, device="cuda")
        cases.append(("norm2", lambda: qsv.qsv_norm2(st, out=nout), state_bytes))
        cases.append(("expval_tfim", lambda: qsv.qsv_expval_zz_x(st, out=nout), state_bytes))
        hout = torch.empty_like(st) if n <= 32 else None   # H psi needs a second state
        if hout is not None:
            cases.append(("apply_tfim", lambda: qsv.qsv_apply_tfim(st, hout), 2 * state_bytes))
        for name, fn, nbytes in cases:
            sec = timed(fn)
            res["%s_%s" % (name, dname)] = {"ms": round(sec * 1e3, 3), "GB/s": round(nbytes / sec / 1e9, 1)}
            _progress("reductions %s %s %.3f ms" % (dname, name, sec * 1e3))
        # a collapse onto one outcome of 4 qubits (reads the kept part, then rewrites the state)
        t0 = time.perf_counter()
        qsv.qsv_collapse(st, [0, 7, 13, n - 1], 5)
        torch.cuda.synchronize()
        res["collapse_r4_%s" % dname] = {"ms": round((time.perf_counter() - t0) * 1e3, 3)}
        del st, hout
        torch.cuda.empty_cache()
    # sampling: 2^20 shots from the 2^20-outcome distribution of a random state's 20 low qubits
    probs = torch.rand(1 << 20, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(2))
    probs /= probs.sum()
    u = torch.rand(1 << 20, dtype=torch.float64, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    sec = timed(lambda: qsv.qsv_sample_cdf(probs, u))
    res["sample_cdf_2^20_shots_2^20_outcomes"] = {"ms": round(sec * 1e3, 3)}
    print(json.dumps({"metric": "reduction and measurement kernels: ms and GB/s", "config": {
        "workload": "random %d-qubit states, complex64 and complex128, %d calls each" % (n, args.steps)},
        "peak_GB/s": HBM_PEAK_GBS, "results": res}), flush=True)


def _sliced_phases(circ, n, m, a):
    """Number of phases the sliced run cuts `circ` into: a gate whose
    non-diagonal targets include global qubits (>= m) makes them active, and
    a phase ends where a gate would need more than `a` active qubits."""
    import numpy as np
    import paper_2203_08826_amd as qsv
    phases, cur = 1, set()
    for g in circ:
        mat = qsv.qsv_gate_matrix(g)
        diag = np.count_nonzero(mat - np.diag(np.diag(mat))) == 0
        need = set() if diag else {q for q in g["targets"] if q >= m}
        if len(cur | need) > a:
            phases += 1
            cur = set(need)
        else:
            cur |= need
    return phases


def workload_sliced(args):
    """A state in pinned host memory run through the device in slices
    (qsv_sliced_run): the n-qubit QFT in complex64 with slices of 2^(n-4)
    amplitudes and two active global qubits, against the same circuit with the
    state resident in HBM; sampled amplitudes checked against the closed form."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    from oracle import statevec as S
    n = args.n
    m, a = n - 4, 2
    circ = W.qft(n)
    x0 = W.basis_index(n, 0)
    t0 = time.perf_counter()
    st = torch.zeros(1 << n, dtype=torch.complex64).pin_memory()
    alloc_s = time.perf_counter() - t0
    _progress("sliced n=%d: pinned %.0f GiB in %.1f s" % (n, st.numel() * 8 / 2**30, alloc_s))
    res = {}
    for mode, name in ((qsv.PLAN_PASSES, "passes"), (qsv.PLAN_PER_GATE, "per_gate")):
        st.zero_()
        st[x0] = 1.0
        t0 = time.perf_counter()
        qsv.qsv_sliced_run(st, circ, m, a, mode=mode)
        sec = time.perf_counter() - t0
        ys = np.random.default_rng(3).integers(0, 1 << n, size=1 << 14)
        err = float(np.max(np.abs(st.numpy()[ys].astype(np.complex128) - S.qft_basis_amplitudes(n, x0, ys))))
        res[name] = {"s": round(sec, 3), "closed_form_max_abs_err": err}
        _progress("sliced %s %.2f s" % (name, sec))
    phases = _sliced_phases(circ, n, m, a)
    link = 2.0 * phases * st.numel() * 8
    for r in res.values():
        r["host_link_GB/s"] = round(link / r["s"] / 1e9, 1)
    del st
    dev = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    dev[x0] = 1.0
    plan = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, jit=1)
    res["in_hbm_compiled_passes_s"] = round(_timed(lambda: qsv.qsv_plan_execute(plan, dev), 1), 4)
    print(json.dumps({"metric": "seconds, state in host memory", "config": {
        "workload": "QFT n=%d complex64 in pinned host memory, slices of 2^%d, %d active global qubits, %d phases" % (
            n, m, a, phases)}, "pinned_alloc_s": round(alloc_s, 1), "host_link_bytes": link, "results": res}), flush=True)


def workload_single_gate(args):
    """Per-gate kernels on their own: dense one-qubit gates on a low, middle
    and high qubit, X, Z, a controlled phase, SWAP and fSim, each timed with
    HIP events on the launch stream over --steps launches, GB/s of touched
    bytes (read + write of the amplitudes the gate changes) and of the
    128-byte lines holding them (complex64 lines hold 16 amplitudes, so a
    gate with a bit below 4 changes part of every line it touches)."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    n = args.n
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    stream = torch.cuda.current_stream()
    res = {}
    for dname, tdt, s in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        st = torch.zeros(1 << n, dtype=tdt, device="cuda")
        st[0] = 1.0
        full = 2.0 * (1 << n) * s
        every = ([], lambda v: True)
        cases = (("H_q0", lambda: qsv.qsv_apply_matrix(st, H, [0]), every),
                 ("H_q3", lambda: qsv.qsv_apply_matrix(st, H, [3]), every),
                 ("H_q12", lambda: qsv.qsv_apply_matrix(st, H, [12]), every),
                 ("H_q%d" % (n - 8), lambda: qsv.qsv_apply_matrix(st, H, [n - 8]), every),
                 ("H_q%d" % (n - 1), lambda: qsv.qsv_apply_matrix(st, H, [n - 1]), every),
                 ("X_q%d" % (n - 1), lambda: qsv.qsv_apply_x(st, n - 1), every),
                 ("Z_q5", lambda: qsv.qsv_apply_z(st, 5), ([5], lambda v: v[0])),
                 ("CU1_c3_t20", lambda: qsv.qsv_apply_phase(st, 20, 0.3, [3]), ([3, 20], lambda v: v[0] and v[1])),
                 ("SWAP_3_20", lambda: qsv.qsv_apply_swap(st, 3, 20), ([3, 20], lambda v: v[0] != v[1])),
                 ("fSim_10_20", lambda: qsv.qsv_apply_fsim(st, 10, 20, 0.4, 0.7), ([10, 20], lambda v: v[0] or v[1])))
        for name, fn, touched in cases:
            nbytes = full * _touched_fraction(*touched)
            lbytes = full * _touched_fraction(*touched, line_bits=(128 // s).bit_length() - 1)
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            e1.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / args.steps
            res["%s_%s" % (name, dname)] = {"ms": round(sec * 1e3, 3), "GB/s": round(nbytes / sec / 1e9, 1),
                                            "frac": round(nbytes / sec / 1e9 / HBM_PEAK_GBS, 4),
                                            "line_GB/s": round(lbytes / sec / 1e9, 1)}
            print("single_gate %s %s %.3f ms %.1f GB/s" % (dname, name, sec * 1e3, nbytes / sec / 1e9), flush=True)
        del st
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "single-gate HBM GB/s (touched bytes)", "config": {
        "workload": "single gates at n=%d, complex64 and complex128, %d launches each" % (n, args.steps)},
        "peak_GB/s": HBM_PEAK_GBS, "results": res}), flush=True)


_HOST_CPUS = None


def host_cpus():
    """(logical CPUs this process may run on, distinct physical cores among
    them), taken once: once OpenMP has bound the main thread (OMP_PROC_BIND)
    the affinity mask shows one CPU."""
    global _HOST_CPUS
    if _HOST_CPUS is not None:
        return _HOST_CPUS
    try:
        allowed = sorted(os.sched_getaffinity(0))
    except AttributeError:
        allowed = list(range(os.cpu_count() or 1))
    cores, cur = {}, {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                continue
            key, val = [x.strip() for x in line.split(":", 1)]
            if key == "processor":
                cur = {"cpu": int(val)}
            elif key in ("physical id", "core id"):
                cur[key] = int(val)
                if "physical id" in cur and "core id" in cur:
                    cores[cur["cpu"]] = (cur["physical id"], cur["core id"])
    except OSError:
        pass
    phys = {cores.get(c, ("cpu", c)) for c in allowed}
    _HOST_CPUS = (len(allowed), max(1, len(phys)))
    return _HOST_CPUS


def pin_oracle_threads():
    """Oracle threads: one per physical core, kept close (before OpenMP starts)."""
    _, phys = host_cpus()
    os.environ.setdefault("OMP_NUM_THREADS", str(phys))
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ.setdefault("OMP_PLACES", "cores")


def host_description():
    """CPU model, logical CPUs and memory of the host the oracle ran on."""
    model, mem_kib = "unknown CPU", 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                mem_kib = int(line.split()[1])
                break
    except OSError:
        pass
    logical, phys = host_cpus()
    return "%s, %d logical CPUs (%d physical cores) available, %.0f GiB RAM" % (model, logical, phys, mem_kib / 2 ** 20)


def exact_qft_infidelity(st, n, x0, chunk=1 << 24):
    """1 - |<QFT|x0>, psi>|^2 / <psi, psi> over all 2^n amplitudes, the exact
    amplitudes exp(2 pi i x0 y / 2^n) / 2^(n/2) formed in float64 chunk by
    chunk on the device (x0 y mod 2^n is exact in int64 for n <= 31)."""
    import torch
    assert n <= 31
    ov = torch.zeros((), dtype=torch.complex128, device=st.device)
    nn = torch.zeros((), dtype=torch.float64, device=st.device)
    for c0 in range(0, 1 << n, chunk):
        y = torch.arange(c0, min(c0 + chunk, 1 << n), dtype=torch.int64, device=st.device)
        ph = ((x0 * y) % (1 << n)).to(torch.float64) * (2.0 * math.pi / (1 << n))
        ex = torch.polar(torch.full_like(ph, 2.0 ** (-n / 2)), ph)
        a = st[c0:c0 + y.numel()].to(torch.complex128)
        ov += torch.sum(torch.conj(ex) * a)
        nn += torch.sum(a.real * a.real + a.imag * a.imag)
    return float(1.0 - (ov.abs() ** 2 / nn).item())


def committed_full_run(n):
    """The committed whole-circuit oracle run of the n-qubit QFT
    (profiles/oracle_qft30_c128_cpu_full_run.md), or None."""
    path = os.path.join(ROOT, "profiles", "oracle_qft%d_c128_cpu_full_run.md" % n)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("full_run_json:"):
            return json.loads(line.split(":", 1)[1])
    return None


def kernel_digest(qsv, plan):
    """First 16 hex digits of the SHA-256 of the generated sources of a plan's
    compiled passes, in launch order (None when it has none): what the
    dominant kernel of a compiled plan is, independent of unrelated edits."""
    import hashlib
    h = hashlib.sha256()
    count = 0
    for i in range(qsv.qsv_plan_stats_get(plan)["n_launches"]):
        if qsv.qsv_plan_op_info(plan, i)["kind"] == 2:
            try:
                src = qsv.qsv_plan_op_source(plan, i)
            except qsv.QsvError:
                return None
            if not src:
                return None   # an interpreted pass
            h.update(src.encode())
            count += 1
    return h.hexdigest()[:16] if count else None


def measured_traffic(kind, digest=None):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary (scaled by the copy-kernel calibration),
    or None when that summary was taken on a different version of the kernel:
    for compiled passes, other generated sources (`digest`, kernel_digest);
    for the interpreted kernel, another version of its source file."""
    files = {"lds_pass": "lds_pass_qft30_c64_traffic.md", "lds_pass_compiled": "lds_pass_compiled_qft30_c64_traffic.md"}
    if kind not in files:
        return None
    import hashlib
    path = os.path.join(ROOT, "profiles", files[kind])
    if not os.path.exists(path):
        return None
    info = None
    for line in open(path):
        if line.startswith("traffic_json:"):
            info = json.loads(line.split(":", 1)[1])
    if info is None:
        return None
    if "kernels_sha256_16" in info:
        if digest != info["kernels_sha256_16"]:
            return None
    else:
        src = os.path.join(ROOT, info["source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if sha != info["source_sha256_16"]:
            return None
    return info["bytes_per_launch"]


def _oracle_seconds(n, circ, psi0, threads=None):
    """Wall seconds of the oracle on a whole circuit (steady clock around the
    gate loop); with `threads` it runs in a child process with that
    OMP_NUM_THREADS (OpenMP fixes its thread count when it starts)."""
    import subprocess
    import numpy as np
    if threads is not None:
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        code = ("import sys, json; sys.path.insert(0, %r); import bench; import workloads as W; "
                "print(json.dumps(bench._oracle_seconds(%d, W.%s, W.random_state(%d, 0))))" % (
                    ROOT, n, "qft(%d)" % n, n))
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
        return json.loads(out.stdout.strip().splitlines()[-1])
    from oracle import statevec as S
    a = np.array(psi0, dtype=np.complex128) if psi0 is not None else S.basis_state(n, 0)
    b = np.empty_like(a)
    t0 = time.perf_counter()
    for g in circ:
        S.apply_gate(a, g, out=b)
        a, b = b, a
    return {"s": time.perf_counter() - t0, "threads": S.num_threads()}


def workload_adiabatic(args):
    """Trotterised adiabatic evolution (Sec. 3.3): H(s) = (1 - s) H0 + s H1
    towards the transverse-field Ising model, second-order steps of RX and ZZ
    phase gates from |+>^n.  Per plan kind: dry run (plan creation with any
    compilation, plus the first execution) and steady seconds, and the final
    energy under H1 from the library's reduction."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    n, T, step = args.n, args.time, args.dt
    circ = W.adiabatic_trotter(n, T=T, dt=step)
    res = {}
    for name, kw in (("per_gate", dict(mode=qsv.PLAN_PER_GATE)), ("passes", dict(mode=qsv.PLAN_PASSES, jit=0)),
                     ("passes_compiled_parametric", dict(mode=qsv.PLAN_PASSES, jit=2))):
        for dname, dt, tdt in (("c64", qsv.QSV_C64, torch.complex64), ("c128", qsv.QSV_C128, torch.complex128)):
            st = torch.full((1 << n,), 2.0 ** (-n / 2), dtype=tdt, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = qsv.qsv_plan_create(n, dt, circ, **kw)
            t1 = time.perf_counter()
            qsv.qsv_plan_execute(plan, st)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            e = float(qsv.qsv_expval_zz_x(st, J=-1.0, h=-1.0, periodic=True).cpu().numpy()[0])
            steady = _timed(lambda: qsv.qsv_plan_execute(plan, st), 2)
            ps = plan.stats()
            res["%s_%s" % (name, dname)] = {"plan_create_s": round(t1 - t0, 3), "dry_run_s": round(t2 - t0, 4),
                                            "steady_s": round(steady, 5), "launches": ps["n_launches"],
                                            "GB/s": round(ps["bytes"] / steady / 1e9, 1), "energy_H1": e}
            print("adiabatic %s %s %s" % (name, dname, json.dumps(res["%s_%s" % (name, dname)])), flush=True)
            del st
            torch.cuda.empty_cache()
    print(json.dumps({"metric": "seconds, dry run and steady", "config": {
        "workload": "adiabatic TFIM evolution n=%d T=%g dt=%g (%d Trotter steps, %d gates), from |+>^n" % (
            n, T, step, int(round(T / step)), len(circ))}, "results": res}), flush=True)


def workload_qft20(args):
    """The plain method on a CPU-checkable size: 20-qubit QFT (220 gates),
    complex128, random Gaussian state (seed 0).  GPU plans: dry run (plan
    creation including compilation, plus the first execution) and steady
    seconds; the oracle on the host cores, all physical cores and one."""
    import numpy as np
    import torch
    import paper_2203_08826_amd as qsv
    import workloads as W
    n = 20
    circ = W.qft(n)
    psi0 = W.random_state(n, 0)
    want = np.fft.ifft(psi0, norm="ortho")   # the QFT of the state (library routine)
    res = {}
    for name, kw in (("per_gate", dict(mode=qsv.PLAN_PER_GATE)), ("passes", dict(mode=qsv.PLAN_PASSES, jit=0)),
                     ("passes_compiled", dict(mode=qsv.PLAN_PASSES, jit=1))):
        st = torch.from_numpy(psi0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, **kw)
        t1 = time.perf_counter()
        qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        err = float(np.max(np.abs(st.cpu().numpy() - want)))
        reps = 20
        t3 = time.perf_counter()
        for _ in range(reps):
            qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        steady = (time.perf_counter() - t3) / reps
        res[name] = {"plan_create_s": round(t1 - t0, 4), "first_execute_s": round(t2 - t1, 5),
                     "dry_run_s": round(t2 - t0, 4), "steady_s": round(steady, 6),
                     "launches": plan.stats()["n_launches"], "max_abs_err_vs_fft": err}
    multi = _oracle_seconds(n, circ, psi0)
    single = _oracle_seconds(n, None, None, threads=1)
    print(json.dumps({"metric": "seconds, dry run and steady (20q QFT c128)", "config": {
        "workload": "QFT n=20 (%d gates), complex128, random Gaussian state seed 0" % len(circ)},
        "gpu": res, "oracle_cpu": {"threads_%d" % multi["threads"]: round(multi["s"], 3),
                                   "threads_1": round(single["s"], 3), "host": host_description()}}), flush=True)


def workload_cpu_baseline_full(args):
    """The oracle on the whole QFT at n qubits (complex128, out of place, from
    the seeded basis state), timed on the host cores, with sampled amplitudes
    checked against the closed form."""
    import numpy as np
    import workloads as W
    from oracle import statevec as S
    n = args.n
    circ = W.qft(n)
    x0 = W.basis_index(n, 0)
    a = S.basis_state(n, x0)
    b = np.empty_like(a)
    per = []
    t0 = time.perf_counter()
    for k, g in enumerate(circ):
        tg = time.perf_counter()
        S.apply_gate(a, g, out=b)
        a, b = b, a
        per.append(time.perf_counter() - tg)
        if k % 40 == 39:
            print("oracle gate %d/%d, %.1f s" % (k + 1, len(circ), time.perf_counter() - t0), flush=True)
    total = time.perf_counter() - t0
    ys = np.random.default_rng(1).integers(0, 1 << n, size=1 << 14)
    err = float(np.max(np.abs(a[ys] - S.qft_basis_amplitudes(n, x0, ys))))
    print(json.dumps({"metric": "oracle seconds, whole circuit", "config": {
        "workload": "QFT n=%d (%d gates), complex128 out of place, basis |x0> seeded" % (n, len(circ))},
        "s": round(total, 2), "per_gate_s": {"mean": round(float(np.mean(per)), 4),
                                             "min": round(float(np.min(per)), 4), "max": round(float(np.max(per)), 4)},
        "threads": S.num_threads(), "omp_proc_bind": os.environ.get("OMP_PROC_BIND", "unset"),
        "closed_form_max_abs_err": err, "host": host_description()}), flush=True)


def stream_calibration(steps):
    """In-place one-shot stream (qsv_scale: one read and one write of every
    amplitude, 16-byte accesses) at a cache-resident size (24 qubits
    complex64 = 128 MiB, inside the 256 MB Infinity Cache) and at HBM sizes
    (30 and 33 qubits complex64, 30 qubits complex128), beside torch's device
    copy: the measured ceilings the gate kernels are compared with."""
    import torch
    import paper_2203_08826_amd as qsv
    stream = torch.cuda.current_stream()
    res = {}
    for n, dt, s in ((24, torch.complex64, 8), (30, torch.complex64, 8), (33, torch.complex64, 8),
                     (30, torch.complex128, 16)):
        a = torch.zeros(1 << n, dtype=dt, device="cuda")
        qsv.qsv_scale(a, -1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            qsv.qsv_scale(a, -1.0)
        e1.record(stream)
        e1.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / steps
        name = "inplace_%dq_%s" % (n, "c64" if s == 8 else "c128")
        res[name] = {"bytes": 2 * (1 << n) * s, "ms": round(sec * 1e3, 4),
                     "GB/s": round(2 * (1 << n) * s / sec / 1e9, 1), "cache_resident": n <= 24}
        if n == 30 and s == 8:
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                b.copy_(a)
            e1.record(stream)
            e1.synchronize()
            sec = e0.elapsed_time(e1) / 1e3 / steps
            res["torch_copy_30q_c64"] = {"bytes": 2 * (1 << n) * s, "ms": round(sec * 1e3, 4),
                                         "GB/s": round(2 * (1 << n) * s / sec / 1e9, 1)}
            del b
        print("calibration %s" % json.dumps({name: res[name]}), flush=True)
        del a
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "in-place stream ceiling GB/s", "peak_GB/s": HBM_PEAK_GBS, "results": res}), flush=True)


def copy_calibration(n, steps):
    """Device-to-device copy of a 2^n complex64 array: the reference kernel
    for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.randn(1 << n, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    nbytes = 2 * a.numel() * 8
    print(json.dumps({"copy_bytes_per_launch": nbytes, "read_bytes": nbytes // 2, "write_bytes": nbytes // 2,
                      "s": dt, "GB/s": round(nbytes / dt / 1e9, 1)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this simulator has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if not args.no_cpu or args.workload in ("cpu_baseline_full", "qft20"):
        pin_oracle_threads()
    import numpy as np
    import torch

    import paper_2203_08826_amd as qsv
    import workloads as W

    if args.copy_calibration:
        copy_calibration(args.n, args.steps)
        return
    if args.stream_calibration:
        stream_calibration(args.steps)
        return
    if args.workload != "qft":
        {"supremacy": workload_supremacy, "variational": workload_variational, "adjoint": workload_adjoint,
         "learned": workload_learned, "single_gate": workload_single_gate, "qft20": workload_qft20,
         "cpu_baseline_full": workload_cpu_baseline_full, "adiabatic": workload_adiabatic,
         "sliced": workload_sliced, "reductions": workload_reductions}[args.workload](args)
        return

    dev = torch.device("cuda:0")
    n = args.n
    circ = W.qft(n)
    x0 = W.basis_index(n, 0)
    modes = {"per_gate": qsv.PLAN_PER_GATE, "greedy": qsv.PLAN_GREEDY, "passes": qsv.PLAN_PASSES,
             "learned": qsv.PLAN_LEARNED}
    model_loaded = False
    if args.plan == "learned" and os.path.exists(args.model):
        from paper_2203_08826_amd import cost_model
        cost_model.load_into_library(args.model)
        model_loaded = True

    stream = torch.cuda.current_stream()

    def basis(dtype):
        st = torch.zeros(1 << n, dtype=dtype, device=dev)
        st[x0] = 1.0
        return st

    def timed_runs(plan, st, steps, warmup):
        t_dry0 = time.perf_counter()
        qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        dry = time.perf_counter() - t_dry0
        for _ in range(warmup):
            qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            qsv.qsv_plan_execute(plan, st)
        torch.cuda.synchronize()
        return dry, (time.perf_counter() - t0) / steps

    # ---------------------------------------------------------- headline plan
    dt = qsv.QSV_C64
    t_create = time.perf_counter()
    plan = qsv.qsv_plan_create(n, dt, circ, mode=modes[args.plan], kmax=args.kmax, jit=args.jit)
    create_s = time.perf_counter() - t_create
    pstats = plan.stats()
    st = basis(torch.complex64)
    # correctness spot check on one fresh application: closed form of QFT|x0>
    t_first = time.perf_counter()
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t_first
    rng = np.random.default_rng(1)
    ys = torch.from_numpy(rng.integers(0, 1 << n, size=1 << 14)).to(dev)
    got = st[ys].cpu().numpy().astype(np.complex128)
    yv = ys.cpu().numpy().astype(np.int64)
    phase = ((x0 * yv) % (1 << n)).astype(np.float64) / float(1 << n)
    want = np.exp(2j * np.pi * phase) / 2 ** (n / 2)
    closed_form_err = float(np.max(np.abs(got - want)))
    c64_state = st.clone()
    infid_exact = exact_qft_infidelity(st, n, x0)
    st = basis(torch.complex64)
    _, step_s = timed_runs(plan, st, args.steps, args.warmup)
    # the paper's dry run: the first execution including compilation
    # (here: plan creation with its kernel compilation, plus the first
    # execution, which loads the code objects)
    dry_s = create_s + first_s
    bytes_plan = pstats["bytes"]

    # ---------------------------------------------------------- dominant kernel roofline (HIP events)
    nops = pstats["n_launches"]
    per_kind = {}
    per_launch_ms = []
    reps = 3
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    for i in range(nops):
        info = qsv.qsv_plan_op_info(plan, i)
        ev0.record(stream)
        for _ in range(reps):
            qsv.qsv_plan_execute_ops(plan, st, i, 1)
        ev1.record(stream)
        ev1.synchronize()
        dur = ev0.elapsed_time(ev1) / 1e3 / reps
        per_launch_ms.append(round(dur * 1e3, 3))
        k = per_kind.setdefault(info["kind"], {"time": 0.0, "count": 0, "bytes": 0.0, "flops": 0.0})
        k["time"] += dur
        k["count"] += 1
        k["bytes"] += info["bytes"]
        k["flops"] += info["flops"]
    kind_names = {0: "gate", 1: "mfma_block", 2: "lds_pass_compiled" if pstats["n_jit_passes"] else "lds_pass",
                  3: "bit_permutation"}
    dom = max(per_kind, key=lambda k: per_kind[k]["time"])
    d = per_kind[dom]
    avg_dur = d["time"] / d["count"]
    bytes_per_launch = d["bytes"] / d["count"]
    achieved = bytes_per_launch / avg_dur / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kind_names[dom], kernel_digest(qsv, plan)),
                "kernel": kind_names[dom], "launches": d["count"], "avg_launch_ms": round(avg_dur * 1e3, 4),
                "bytes_per_launch": bytes_per_launch, "per_launch_ms": per_launch_ms}

    # ---------------------------------------------------------- comparison plans
    compare = {}
    infid = None
    if not args.no_baselines:
        del st
        torch.cuda.empty_cache()
        for name, mode, cdt, tdt, steps in (("plain_c128", qsv.PLAN_PER_GATE, qsv.QSV_C128, torch.complex128, 2),
                                            ("per_gate_c64", qsv.PLAN_PER_GATE, qsv.QSV_C64, torch.complex64, 2),
                                            ("greedy2_c64", qsv.PLAN_GREEDY, qsv.QSV_C64, torch.complex64, 2),
                                            ("passes_interpreted_c64", qsv.PLAN_PASSES, qsv.QSV_C64, torch.complex64, 3)):
            p2 = qsv.qsv_plan_create(n, cdt, circ, mode=mode, kmax=2)
            s2 = basis(tdt)
            if name == "plain_c128":
                qsv.qsv_plan_execute(p2, s2)
                ref = s2.clone()
                a = c64_state.to(torch.complex128)
                ov = qsv.qsv_inner(ref, a).cpu().numpy()
                n1 = qsv.qsv_norm2(ref).cpu().numpy()[0]
                n2 = qsv.qsv_norm2(a).cpu().numpy()[0]
                infid = float(1.0 - (ov[0] ** 2 + ov[1] ** 2) / (n1 * n2))
                del ref, a
                s2 = basis(tdt)
            dry2, t2 = timed_runs(p2, s2, steps, 0)
            b2 = p2.stats()["bytes"]
            compare[name] = {"s": round(t2, 5), "GB/s": round(b2 / t2 / 1e9, 1), "bytes": b2}
            del s2
            torch.cuda.empty_cache()
        compare["plain_c128_over_headline"] = round(compare["plain_c128"]["s"] / step_s, 2)

    # ---------------------------------------------------------- oracle on host cores
    cpu = None
    if not args.no_cpu:
        from oracle import statevec as S
        a = S.basis_state(n, x0)
        b = np.empty_like(a)
        k = 0
        t0 = time.perf_counter()
        while k < len(circ) and time.perf_counter() - t0 < args.cpu_seconds:
            S.apply_gate(a, circ[k], out=b)
            a, b = b, a
            k += 1
        dt_cpu = time.perf_counter() - t0
        per_gate = dt_cpu / k
        cpu = {"value": round(per_gate * len(circ), 2), "unit": "s", "cores": S.num_threads(), "kind": "oracle",
               "sample": "first %d gates of the %d-qubit QFT (complex128, out of place, OMP_PROC_BIND=%s), %.2f s "
                         "measured; value = mean seconds per gate x %d gates" % (
                             k, n, os.environ.get("OMP_PROC_BIND", "unset"), dt_cpu, len(circ)),
               "host": host_description()}
        full = committed_full_run(n)
        if full is not None:   # the whole circuit, run once on this machine's host (cross-check)
            cpu["full_run_s"] = full["s"]
            cpu["full_run_threads"] = full["threads"]
        del a, b

    gbps = bytes_plan / step_s / 1e9
    out = {
        "metric": "circuit s & HBM GB/s, 30q QFT c64; fused+learned vs plain c128 at infid<=1e-6",
        "value": round(step_s, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "QFT n=%d (%d gates), complex64 state from basis |x0>, x0 seeded" % (n, len(circ)),
                   "plan": args.plan, "plan_used": pstats["mode_used"], "model_loaded": model_loaded,
                   "launches": pstats["n_launches"], "passes": pstats["n_passes"],
                   "compiled_passes": pstats["n_jit_passes"]},
        "plan_create_s": round(create_s, 3),
        "hbm_gbps": round(gbps, 1),
        "hbm_frac": round(gbps / HBM_PEAK_GBS, 4),
        "plan_bytes": bytes_plan,
        "dry_run_s": round(dry_s, 5),
        "first_execute_s": round(first_s, 5),
        "closed_form_max_abs_err": closed_form_err,
        "infidelity_c64_vs_exact_all_amplitudes": infid_exact,
        "infidelity_c64_vs_c128": infid,
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
