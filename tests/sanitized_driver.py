"""Host-side workout of libqsv for the AddressSanitizer / UndefinedBehavior-
Sanitizer build (run by test_sanitized_host.py in a child process with the
sanitizer runtime preloaded and QSV_LIBRARY naming that build).

Everything here stays on the host: argument validation and its error paths
(overlapping output ranges among them),
group enumeration, gate matrices, and plan creation in every mode that needs
no device (per-gate, greedy fusion with and without matrix-core blocks, LDS
passes interpreted and compiled, the density-matrix doubling), with every
op's description read back.  A sanitizer report ends the process with a
non-zero status."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_2203_08826_amd as qsv  # noqa: E402
import workloads as W  # noqa: E402


def expect_error(fn, *a, **k):
    try:
        fn(*a, **k)
    except qsv.QsvError:
        return
    raise AssertionError("no error from %s%r" % (fn.__name__, a))


def read_back(p):
    st = p.stats()
    for i in range(st["n_launches"]):
        qsv.qsv_plan_op_info(p, i)
        qsv.qsv_plan_op_gates(p, i)
        qsv.qsv_plan_op_features(p, i)
        for fn in (qsv.qsv_plan_op_program, qsv.qsv_plan_op_source):
            try:
                fn(p, i)
            except qsv.QsvError:
                pass   # not an LDS pass, or not a compiled one
    try:
        qsv.qsv_plan_blocks(p)
    except qsv.QsvError:
        pass   # plans without fusion blocks say so
    return st


def main():
    count = 0
    # validation
    for n, t, c in ((0, [0], []), (70, [0], []), (5, [5], []), (5, [1, 1], []), (5, [1], [1]), (5, [-1], [])):
        assert qsv.qsv_validate(n, qsv.QSV_C64, t, c) != 0
    assert qsv.qsv_validate(5, qsv.QSV_C64, [4, 0], [2]) == 0
    expect_error(qsv.qsv_plan_create, 4, qsv.QSV_C64, [W.gate("H", [4])])
    expect_error(qsv.qsv_plan_create, 12, qsv.QSV_C64, W.qft(12), mode=qsv.PLAN_PASSES, jit=3)
    expect_error(qsv.qsv_plan_create, 12, qsv.QSV_C64, W.qft(12), mode=qsv.PLAN_GREEDY, kmax=9)
    # group enumeration
    for n, bits in ((6, [0]), (9, [2, 5, 8]), (12, [0, 3, 6, 11])):
        qsv.qsv_group_index_host(n, bits, 0, 1 << (n - len(bits)))
        qsv.qsv_group_index_host(n, bits, 3, 2)
    expect_error(qsv.qsv_group_index_host, 9, [8, 2], 0, 4)
    # gate matrices
    rng = np.random.default_rng(0)
    for g in W.random_circuit(6, 120, seed=1, kmax=4, max_controls=2):
        qsv.qsv_gate_matrix(g)
    # plans
    for n in (1, 2, 3, 5, 8, 12, 15):
        circs = [[], W.random_circuit(n, 60, seed=n, kmax=min(3, n), max_controls=min(2, n - 1))]
        if n >= 2:
            circs.append(W.qft(n))
        if n >= 4:
            circs += [W.supremacy(n, 4, seed=n), W.variational(n, 2, seed=n)]
        for circ in circs:
            for dt in (qsv.QSV_C64, qsv.QSV_C128):
                kinds = [dict(mode=qsv.PLAN_PER_GATE), dict(mode=qsv.PLAN_LEARNED)]
                kinds += [dict(mode=qsv.PLAN_GREEDY, kmax=k, use_mfma=m) for k in range(1, 7) for m in (0, 1)]
                kinds += [dict(mode=qsv.PLAN_PASSES, jit=j) for j in (0, 1, 2)] if n >= 5 else []
                for kw in kinds:
                    try:
                        p = qsv.qsv_plan_create(n, dt, circ, **kw)
                    except qsv.QsvError:
                        continue   # a documented refusal (say, a block wider than the register)
                    read_back(p)
                    del p
                    count += 1
    for n in (2, 3, 5):
        p = qsv.qsv_dm_plan_create(n, qsv.QSV_C128, W.random_circuit(n, 20, seed=3, kmax=2, max_controls=1))
        read_back(p)
        count += 1
    rng.standard_normal(1)
    # outputs overlapping the state they are computed from: refused before any
    # device work (fake, never dereferenced addresses)
    import ctypes
    lib = qsv.load()
    base = 1 << 20
    qs = (ctypes.c_int * 2)(0, 3)
    assert lib.qsv_apply_tfim(ctypes.c_void_p(base), ctypes.c_void_p(base + 512), 10, qsv.QSV_C64,
                              ctypes.c_double(1.0), ctypes.c_double(0.5), 0, None) == -10
    assert lib.qsv_probabilities(ctypes.c_void_p(base), 10, qsv.QSV_C64, qs, 2, ctypes.c_void_p(base + 4096), None) == -10
    assert lib.qsv_collapse(ctypes.c_void_p(base), 10, qsv.QSV_C128, qs, 2, ctypes.c_uint64(1),
                            ctypes.c_void_p(base + 16 * 1023), None) == -10
    assert lib.qsv_adjoint_grad(ctypes.c_void_p(base), ctypes.c_void_p(base + 4096), 10, qsv.QSV_C64, None, 0,
                                None, None) == -10
    print("sanitized host workout: %d plans" % count, flush=True)


if __name__ == "__main__":
    main()
