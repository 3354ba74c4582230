"""Host-side checks of libqsv.so that need no GPU: symbols, validation,
index generation and the library's own gate matrices."""
import os
import re

import numpy as np
import pytest

import paper_2203_08826_amd as qsv
import workloads as W
from oracle import gates as OG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "qsv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = qsv.load()
    syms = _declared_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(lib, s), s
        assert s in qsv._abi.SIGNATURES, s
    assert qsv.qsv_abi_version() == 2


def test_validation_codes():
    ok = qsv.qsv_validate(5, qsv.QSV_C64, [0, 3], [4])
    assert ok == 0
    assert qsv.qsv_validate(0, 0, [0], []) == -3
    assert qsv.qsv_validate(41, 0, [0], []) == -3
    assert qsv.qsv_validate(5, 2, [0], []) == -2
    assert qsv.qsv_validate(5, 0, [5], []) == -4
    assert qsv.qsv_validate(5, 0, [-1], []) == -4
    assert qsv.qsv_validate(5, 0, [1, 1], []) == -5
    assert qsv.qsv_validate(5, 0, [1], [1]) == -5
    assert qsv.qsv_validate(3, 0, [0, 1], [2, 3]) == -6
    assert qsv.qsv_validate(10, 0, list(range(7)), []) == -6
    assert qsv.qsv_status_string(-5) == "repeated qubit"


def test_errors_leave_no_launch_and_raise():
    # validation runs before any HIP call, so it works without a GPU
    import ctypes
    lib = qsv.load()
    t = (ctypes.c_int * 1)(7)
    st = lib.qsv_apply_x(ctypes.c_void_p(16), 5, 0, 7, None, 0, None)
    assert st == -4 and "outside" in qsv.qsv_last_error()
    st = lib.qsv_apply_x(None, 5, 0, 1, None, 0, None)
    assert st == -1
    st = lib.qsv_apply_x(ctypes.c_void_p(8), 5, 0, 1, None, 0, None)
    assert st == -7
    del t


@pytest.mark.parametrize("n", [1, 3, 7, 12])
def test_group_index_is_a_bijection_onto_disjoint_groups(n):
    rng = np.random.default_rng(n)
    for m in range(0, min(n, 4) + 1):
        bits = sorted(int(b) for b in rng.permutation(n)[:m])
        base = qsv.qsv_group_index_host(n, bits, 0, 1 << (n - m))
        mask = sum(1 << b for b in bits)
        assert np.all((base & np.uint64(mask)) == 0)
        # groups {base + sub-mask of bits} tile [0, 2^n) exactly once
        seen = np.zeros(1 << n, dtype=np.int64)
        subs = [sum(1 << bits[j] for j in range(m) if (s >> j) & 1) for s in range(1 << m)]
        for s in subs:
            np.add.at(seen, (base + np.uint64(s)).astype(np.int64), 1)
        assert np.all(seen == 1)
        # the paper's one-qubit formula i1 = ((g >> t) << (t + 1)) + (g & (2^t - 1))
        if m == 1:
            g = np.arange(1 << (n - 1), dtype=np.uint64)
            t = np.uint64(bits[0])
            want = ((g >> t) << (t + np.uint64(1))) + (g & ((np.uint64(1) << t) - np.uint64(1)))
            assert np.array_equal(base, want)


def test_library_gate_matrices_match_oracle():
    rng = np.random.default_rng(0)
    names = ["H", "X", "Y", "Z", "SX", "SY", "SW", "RX", "RY", "RZ", "U1", "CNOT", "CZ", "CU1", "SWAP", "FSIM"]
    for name in names:
        for _ in range(3):
            k = 2 if name in ("SWAP", "FSIM") else 1
            g = W.gate(name, list(range(k)), [], list(rng.uniform(0, 2 * np.pi, size=2)))
            got = qsv.qsv_gate_matrix(g)
            want = OG.target_matrix(dict(g, params=g["params"][:1] if name not in ("FSIM",) else g["params"]))
            assert np.max(np.abs(got - want)) <= 1e-15, name
    u = W.random_unitary(3, rng)
    g = {"name": "UNITARY", "targets": [0, 1, 2], "controls": [], "matrix": u}
    assert np.array_equal(qsv.qsv_gate_matrix(g), u)
    d = W.random_phases(2, rng)
    g = {"name": "DIAG", "targets": [0, 1], "controls": [], "diag": d}
    assert np.array_equal(qsv.qsv_gate_matrix(g), np.diag(d))


def test_pass_compilation_on_host():
    """jit=1 compiles every LDS pass at plan creation with the host compiler
    only (no device needed); the generated source turns permutation rows into
    plain moves and keeps the interpreted program's op sequence."""
    n = 12
    circ = W.qft(n)
    p = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, jit=1)
    st = p.stats()
    assert st["n_passes"] >= 1 and st["n_jit_passes"] >= 1
    src = qsv.qsv_plan_op_source(p, 0)
    assert 'extern "C" __global__' in src and "qsv_pass_jit" in src
    # an X on a local qubit: both rows are single unit entries -> moves only
    px = qsv.qsv_plan_create(n, qsv.QSV_C128, [W.gate("X", [11])], mode=qsv.PLAN_PASSES)
    sx = qsv.qsv_plan_op_source(px, 0)
    moves = [l for l in sx.splitlines() if "v[" in l and ".x =" in l]
    assert moves and all("*" not in l for l in moves)
    # the interpreted plan of the same circuit is left without compiled passes
    assert qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES).stats()["n_jit_passes"] == 0


def test_parametric_passes_depend_only_on_structure():
    """jit=2: matrices and angles are read from the program, so two circuits
    that differ only in their angles compile to the same kernel sources, and
    the second plan finds every kernel compiled already (re-binding the
    angles of an ansatz costs host planning only)."""
    import time
    n = 14
    a = qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 3, seed=1), mode=qsv.PLAN_PASSES, jit=2)
    t0 = time.perf_counter()
    b = qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 3, seed=2), mode=qsv.PLAN_PASSES, jit=2)
    assert time.perf_counter() - t0 < 2.0   # a compilation takes seconds
    na = a.stats()["n_launches"]
    assert na == b.stats()["n_launches"] and a.stats()["n_jit_passes"] == na
    sa = [qsv.qsv_plan_op_source(a, i) for i in range(na)]
    assert sa == [qsv.qsv_plan_op_source(b, i) for i in range(na)]
    # literal kernels (jit=1) differ with the angles
    c = qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 1, seed=1), mode=qsv.PLAN_PASSES, jit=1)
    d = qsv.qsv_plan_create(n, qsv.QSV_C64, W.variational(n, 1, seed=2), mode=qsv.PLAN_PASSES, jit=1)
    assert qsv.qsv_plan_op_source(c, 0) != qsv.qsv_plan_op_source(d, 0)
    with pytest.raises(qsv.QsvError):
        qsv.qsv_plan_create(n, qsv.QSV_C64, W.qft(n), mode=qsv.PLAN_PASSES, jit=3)


def test_final_permutation_folds_only_when_it_saves_a_sweep():
    n = 20
    circ = [W.gate("H", [q]) for q in range(4)] + [W.gate("SWAP", [i, n - 1 - i]) for i in range(n // 2)]
    kinds = lambda p: [qsv.qsv_plan_op_info(p, i)["kind"] for i in range(p.stats()["n_launches"])]
    assert kinds(qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, local_bits=12)) == [2, 3]
    assert kinds(qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, local_bits=12, jit=1)) == [2]
    # the 30-qubit QFT would need one more pass to fold its reversal: it stays a separate sweep,
    # the permutation kernel when interpreted, a gate-free compiled pass when compiled
    qi = qsv.qsv_plan_create(30, qsv.QSV_C64, W.qft(30), mode=qsv.PLAN_PASSES, local_bits=12)
    assert kinds(qi) == [2, 2, 2, 2, 3]
    qc = qsv.qsv_plan_create(30, qsv.QSV_C64, W.qft(30), mode=qsv.PLAN_PASSES, local_bits=12, jit=1)
    assert kinds(qc) == [2, 2, 2, 2, 2] and qc.stats()["n_jit_passes"] == 5


def _no_swaps(circ):
    return [g for g in circ if not (g["name"] == "SWAP" and not g.get("controls"))]


@pytest.mark.parametrize("name,n,jit", [("supremacy", 14, 0), ("variational", 13, 0), ("random", 14, 0), ("random3", 16, 0),
                                        ("supremacy", 16, 1)])
def test_pass_planner_reorders_only_commuting_gates(name, n, jit):
    """The pass planner lets a gate join an open pass ahead of earlier gates
    it commutes with.  The ops' gate lists form a reordering of the circuit,
    and the oracle applied in that order gives the circuit's state."""
    from oracle import statevec as S
    circ = {"supremacy": lambda: W.supremacy(n, 8, seed=3),
            "variational": lambda: W.variational(n, 4, seed=3),
            "random": lambda: _no_swaps(W.random_circuit(n, 300, seed=3, kmax=2, max_controls=1)),
            "random3": lambda: _no_swaps(W.random_circuit(n, 300, seed=4, kmax=3, max_controls=2))}[name]()
    p = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES, local_bits=10 if jit else 9, jit=jit)
    order = [i for k in range(p.stats()["n_launches"]) for i in qsv.qsv_plan_op_gates(p, k)]
    assert sorted(order) == list(range(len(circ)))
    assert order != sorted(order)   # something moved
    psi0 = W.random_state(n, 7)
    want = S.run_circuit(psi0, circ)
    got = S.run_circuit(psi0, [circ[i] for i in order])
    assert np.max(np.abs(got - want)) <= 1e-12


def test_lookahead_respects_non_commuting_gates():
    """A phase gate may pass a skipped gate only where both act diagonally:
    Z on q0 passes a skipped CZ(q11, q0) but not a skipped H on q0's partner
    path; a gate on a skipped gate's target waits."""
    n = 12
    circ = [W.gate("H", [q]) for q in range(9)]           # fills the 9 local bits
    circ += [W.gate("H", [11])]                           # 9: does not fit -> skipped
    circ += [W.gate("CZ", [0], [11])]                     # 10: diagonal on 11, skipped H is not -> blocked
    circ += [W.gate("Z", [0])]                            # 11: 0 is diagonal-blocked only -> joins
    circ += [W.gate("H", [0])]                            # 12: 0 is blocked by the CZ -> waits
    circ += [W.gate("RZ", [3], [], [0.4]), W.gate("H", [4])]   # 13, 14: untouched qubits -> join
    p = qsv.qsv_plan_create(n, qsv.QSV_C128, circ, mode=qsv.PLAN_PASSES, local_bits=9)
    first = qsv.qsv_plan_op_gates(p, 0)
    assert first == list(range(9)) + [11, 13, 14]
    from oracle import statevec as S
    order = [i for k in range(p.stats()["n_launches"]) for i in qsv.qsv_plan_op_gates(p, k)]
    psi0 = W.random_state(n, 1)
    assert np.max(np.abs(S.run_circuit(psi0, [circ[i] for i in order]) - S.run_circuit(psi0, circ))) <= 1e-12


def _lambda_body(src, head, tail):
    i = src.index(head) + len(head)
    return src[i:src.index(tail, i)]


def _c_expr(e):
    return re.sub(r"(0x[0-9a-f]+|\d+)ull", r"\1", e)


@pytest.mark.parametrize("n,circ_kind", [(16, "reversal"), (17, "mixed")])
def test_chunk_pair_enumeration_covers_each_pair_once(n, circ_kind):
    """A compiled pass that stores its result permuted pairs chunk c with
    chunk sigma(c); its work items enumerate one representative per pair
    (and every chunk sigma fixes), which the generated index maps must
    cover exactly once."""
    if circ_kind == "reversal":
        circ = [W.gate("H", [0])] + [W.gate("SWAP", [i, n - 1 - i]) for i in range(n // 2)]
    else:   # some non-local bits fixed, some paired
        circ = [W.gate("H", [0])] + [W.gate("SWAP", [a, b]) for a, b in [(0, 15), (1, 14), (12, 16), (3, 4)]]
    p = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PASSES, local_bits=12, jit=1)
    src = [qsv.qsv_plan_op_source(p, k) for k in range(p.stats()["n_launches"])]
    src = [s for s in src if "pair_base" in s]
    assert src, "no chunk-pair pass"
    s = src[0]
    body = _lambda_body(s, "auto pair_base = [&](unsigned long long w) {", " return 0ull; };")
    groups = re.findall(r"if \(w < (\w+)\) \{ const unsigned long long r = w - (\w+); \(void\)r; return ([^;]+); \}", body)
    groups = [(int(_c_expr(a), 0), int(_c_expr(b), 0), _c_expr(e)) for a, b, e in groups]
    part = _c_expr(_lambda_body(s, "auto partner = [&](unsigned long long b) { return ", "; };"))
    partner = eval("lambda b: " + part)
    items = groups[-1][0]
    seen = set()
    for w in range(items):
        for end, start, e in groups:
            if w < end:
                base = eval(e, {"r": w - start})
                break
        pb = partner(base)
        assert partner(pb) == base
        key = (min(base, pb), max(base, pb))
        assert key not in seen, (w, base, pb)
        seen.add(key)
    # every chunk appears in exactly one pair: 2 * pairs + fixed = chunks
    chunks = {b for k in seen for b in k}
    L = 12
    assert len(chunks) == 1 << (n - L)


def test_op_gates_of_per_gate_and_greedy_plans():
    """qsv_plan_op_gates on the other planners: one gate per op in circuit
    order for per-gate plans; the greedy blocks' members for fused plans."""
    n = 10
    circ = W.random_circuit(n, 80, seed=5, kmax=2, max_controls=1)
    p = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_PER_GATE)
    assert [qsv.qsv_plan_op_gates(p, k) for k in range(p.stats()["n_launches"])] == [[i] for i in range(len(circ))]
    g = qsv.qsv_plan_create(n, qsv.QSV_C64, circ, mode=qsv.PLAN_GREEDY, kmax=3)
    ops = [qsv.qsv_plan_op_gates(g, k) for k in range(g.stats()["n_launches"])]
    assert sorted(i for o in ops for i in o) == list(range(len(circ)))
    blocks = qsv.qsv_plan_blocks(g)
    for b, members in enumerate(ops):
        assert all(blocks[i] == b for i in members)


def test_memory_stats_on_the_host():
    """qsv_memory_stats is host-only: the peak never falls below the
    current total, and a reset brings the peak down to it."""
    cur, peak = qsv.qsv_memory_stats()
    assert peak >= cur >= 0
    cur2, peak2 = qsv.qsv_memory_stats(reset_peak=True)
    assert cur2 == cur
    assert qsv.qsv_memory_stats() == (cur, cur)


def _exchange_program(blob):
    """(load partition, [partitions after each exchange]) of a serialised pass
    program: header, partitions of 5 register + 9 thread positions, ops of
    112 bytes whose kind 1 is an exchange to partition `a`."""
    import struct
    L, nops, npart, load_part = struct.unpack_from("<4i", blob, 0)
    off_part, off_ops = struct.unpack_from("<2i", blob, 240)
    parts = [(list(struct.unpack_from("<5i", blob, off_part + 56 * q)),
              list(struct.unpack_from("<9i", blob, off_part + 56 * q + 20))) for q in range(npart)]
    seq = []
    for o in range(nops):
        kind, a = struct.unpack_from("<2i", blob, off_ops + 112 * o)
        if kind == 1:
            seq.append(a)
    return parts, load_part, seq


def _local_index(part, t, j, RB, TB):
    reg, thr = part
    return sum(((j >> i) & 1) << reg[i] for i in range(RB)) | sum(((t >> u) & 1) << thr[u] for u in range(TB))


@pytest.mark.parametrize("dt", [qsv.QSV_C64, qsv.QSV_C128])
def test_compiled_exchanges_realise_their_partitions(dt):
    """Every LDS statement of the compiled passes (split or not) simulated for
    every lane: after the exchanges a lane's registers hold exactly the
    amplitudes the program's last partition assigns them (partitions read
    from the serialised program, addresses from the generated source)."""
    import re

    def swz(l):
        return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15)

    checked = split_seen = 0
    for circ in (W.qft(20), W.supremacy(20, 8, seed=1), W.random_circuit(20, 150, seed=4)):
        p = qsv.qsv_plan_create(20, dt, circ, mode=qsv.PLAN_PASSES, jit=1)
        for i in range(p.stats()["n_launches"]):
            if qsv.qsv_plan_op_info(p, i)["kind"] != 2:   # not an LDS pass
                continue
            src = qsv.qsv_plan_op_source(p, i)
            parts, load_part, seq = _exchange_program(qsv.qsv_plan_op_program(p, i))
            if not seq:
                continue
            NR = int(re.search(r"    C v\[(\d+)\];", src).group(1))
            RB = NR.bit_length() - 1
            T = int(re.search(r"(?:__launch_bounds__|amdgpu_flat_work_group_size)\((\d+)", src).group(1))
            TB = T.bit_length() - 1
            csz = 8 if dt == qsv.QSV_C64 else 16
            offs = {}
            for name, expr in re.findall(r"const unsigned (x[owr]\d+) = swz\((.*?)\) \* \(unsigned\)sizeof\(C\);", src):
                pairs = [(int(u), int(q)) for u, q in re.findall(r"\(\(t >> (\d+)\) & 1u\) << (\d+)\)", expr)]
                offs[name] = [swz(sum(((t >> u) & 1) << q for u, q in pairs)) * csz for t in range(T)]
            v = [[_local_index(parts[load_part], t, j, RB, TB) for j in range(NR)] for t in range(T)]
            xt = None
            lds = {}
            body = src[src.index("auto run_ops"):]
            pat = re.compile(r"\*\(C \*\)\(\(char \*\)lds \+ \((x[ow]\d+) \^ (\d+)u\)\) = v\[(\d+)\];|"
                             r"(v|xt)\[(\d+)\] = \*\(const C \*\)\(\(const char \*\)lds \+ \((x[or]\d+) \^ (\d+)u\)\);|"
                             r"\{ C xt\[\d+\];|v\[(\d+)\] = xt\[(\d+)\];")
            cond_pat = re.compile(r"^\s*if \(\(\(t >> (\d+)\) & 1u\) == (\d+)u\) \{")
            for line in body.splitlines():
                # a round of a split exchange may be limited to the threads
                # with one bit of their index 0 (then 1): one line per round
                cm = cond_pat.match(line)
                ts = [t for t in range(T) if not cm or ((t >> int(cm.group(1))) & 1) == int(cm.group(2))]
                for m in pat.finditer(line):
                    if m.group(0).startswith("{ C xt"):
                        xt = [[None] * NR for _ in range(T)]
                        split_seen += 1
                    elif m.group(1):
                        o, c, j = offs[m.group(1)], int(m.group(2)), int(m.group(3))
                        for t in ts:
                            lds[o[t] ^ c] = v[t][j]
                    elif m.group(4):
                        dst, j, o, c = m.group(4), int(m.group(5)), offs[m.group(6)], int(m.group(7))
                        for t in ts:
                            (v if dst == "v" else xt)[t][j] = lds[o[t] ^ c]
                    else:
                        j, k = int(m.group(8)), int(m.group(9))
                        for t in ts:
                            v[t][j] = xt[t][k]
            final = parts[seq[-1]]
            assert all(v[t][j] == _local_index(final, t, j, RB, TB) for t in range(T) for j in range(NR)), (i, circ[0])
            checked += 1
    assert checked >= 4
    if dt == qsv.QSV_C64:
        assert split_seen >= 1


def test_apply_tfim_rejects_overlapping_states_on_the_host():
    """H psi writes out while it still reads state: overlapping ranges are
    refused before anything is queued (no device is touched)."""
    import ctypes
    lib = qsv.load()
    base = 1 << 20   # an aligned address; never dereferenced
    for off in (0, 64, -64):
        st = lib.qsv_apply_tfim(ctypes.c_void_p(base), ctypes.c_void_p(base + off * 8), 10, qsv.QSV_C64,
                                ctypes.c_double(1.0), ctypes.c_double(0.5), 0, None)
        assert st == -10, (off, st)   # QSV_ERR_ARG


def test_outputs_overlapping_their_inputs_are_refused_on_the_host():
    """Probabilities, collapse and the adjoint write device outputs while they
    still read the state: an output range inside the state is refused before
    anything is queued (fake, never dereferenced addresses)."""
    import ctypes
    lib = qsv.load()
    base = 1 << 20
    n = 10
    qs = (ctypes.c_int * 2)(0, 3)
    for fn in (lib.qsv_probabilities, lib.qsv_probabilities_noalloc):
        st = fn(ctypes.c_void_p(base), n, qsv.QSV_C64, qs, 2, ctypes.c_void_p(base + 4096), None)
        assert st == -10, st
    st = lib.qsv_collapse(ctypes.c_void_p(base), n, qsv.QSV_C128, qs, 2, ctypes.c_uint64(1),
                          ctypes.c_void_p(base + 16 * 1023), None)
    assert st == -10, st
    st = lib.qsv_adjoint_grad(ctypes.c_void_p(base), ctypes.c_void_p(base + 8 * 512), n, qsv.QSV_C64, None, 0,
                              None, None)
    assert st == -10, st
