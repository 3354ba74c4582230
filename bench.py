"""Benchmark: 30-qubit QFT, complex64, on one MI355X.

A step is one application of the whole QFT circuit (n H gates, n(n-1)/2
controlled phases, n/2 SWAPs) to a 2^n complex64 state resident in HBM,
with the plan the library picks (LDS passes scored by the cost model when
one is loaded).  Also reported: the same circuit as plain per-gate
complex128 and per-gate / greedy-fused complex64, the complex64 state's
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--plan", default="passes", choices=["per_gate", "greedy", "passes", "learned"])
    ap.add_argument("--kmax", type=int, default=2)
    ap.add_argument("--no-baselines", action="store_true", help="skip the per-gate / c128 comparison plans")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-gates", type=int, default=4, help="oracle sample: first gates of the circuit")
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2203_08826_amd", "cost_model.npz"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain device copy of 2^n complex64 (HBM ceiling and counter calibration)")
    return ap.parse_args()


def copy_calibration(n, steps):
    """Device-to-device copy of a 2^n complex64 array: the measured HBM
    ceiling, and the reference kernel for scaling FETCH_SIZE / WRITE_SIZE."""
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

    import numpy as np
    import torch

    import paper_2203_08826_amd as qsv
    import workloads as W

    if args.copy_calibration:
        copy_calibration(args.n, args.steps)
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
    plan = qsv.qsv_plan_create(n, dt, circ, mode=modes[args.plan], kmax=args.kmax)
    pstats = plan.stats()
    st = basis(torch.complex64)
    # correctness spot check on one fresh application: closed form of QFT|x0>
    qsv.qsv_plan_execute(plan, st)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    ys = torch.from_numpy(rng.integers(0, 1 << n, size=1 << 14)).to(dev)
    got = st[ys].cpu().numpy().astype(np.complex128)
    yv = ys.cpu().numpy().astype(np.int64)
    phase = ((x0 * yv) % (1 << n)).astype(np.float64) / float(1 << n)
    want = np.exp(2j * np.pi * phase) / 2 ** (n / 2)
    closed_form_err = float(np.max(np.abs(got - want)))
    c64_state = st.clone()
    st = basis(torch.complex64)
    dry_s, step_s = timed_runs(plan, st, args.steps, args.warmup)
    bytes_plan = pstats["bytes"]

    # ---------------------------------------------------------- dominant kernel roofline (HIP events)
    nops = pstats["n_launches"]
    per_kind = {}
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
        k = per_kind.setdefault(info["kind"], {"time": 0.0, "count": 0, "bytes": 0.0, "flops": 0.0})
        k["time"] += dur
        k["count"] += 1
        k["bytes"] += info["bytes"]
        k["flops"] += info["flops"]
    kind_names = {0: "gate", 1: "mfma_block", 2: "lds_pass"}
    dom = max(per_kind, key=lambda k: per_kind[k]["time"])
    d = per_kind[dom]
    avg_dur = d["time"] / d["count"]
    bytes_per_launch = d["bytes"] / d["count"]
    achieved = bytes_per_launch / avg_dur / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kind_names[dom], "launches": d["count"], "avg_launch_ms": round(avg_dur * 1e3, 4),
                "bytes_per_launch": bytes_per_launch}

    # ---------------------------------------------------------- comparison plans
    compare = {}
    infid = None
    if not args.no_baselines:
        del st
        torch.cuda.empty_cache()
        for name, mode, cdt, tdt, steps in (("plain_c128", qsv.PLAN_PER_GATE, qsv.QSV_C128, torch.complex128, 2),
                                            ("per_gate_c64", qsv.PLAN_PER_GATE, qsv.QSV_C64, torch.complex64, 2),
                                            ("greedy2_c64", qsv.PLAN_GREEDY, qsv.QSV_C64, torch.complex64, 2)):
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
        k = args.cpu_gates
        a = S.basis_state(n, x0)
        b = np.empty_like(a)
        t0 = time.perf_counter()
        for g in circ[:k]:
            S.apply_gate(a, g, out=b)
            a, b = b, a
        dt_cpu = time.perf_counter() - t0
        per_gate = dt_cpu / k
        cpu = {"value": round(per_gate * len(circ), 2), "unit": "s", "cores": S.num_threads(), "kind": "oracle",
               "sample": "first %d gates of the %d-qubit QFT (complex128, out of place), %.2f s measured; "
                         "value = mean seconds per gate x %d gates" % (k, n, dt_cpu, len(circ))}
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
                   "launches": pstats["n_launches"], "passes": pstats["n_passes"]},
        "hbm_gbps": round(gbps, 1),
        "hbm_frac": round(gbps / HBM_PEAK_GBS, 4),
        "plan_bytes": bytes_plan,
        "dry_run_s": round(dry_s, 5),
        "closed_form_max_abs_err": closed_form_err,
        "infidelity_c64_vs_c128": infid,
        "compare": compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
