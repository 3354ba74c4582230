"""Oracle greedy gate fusion and circuit depth.  Test infrastructure only.

Gate fusion section of the benchmarks (Sec. 3.2): the circuit's gates are
walked in order and one- and two-qubit gates acting on the same qubits are
greedily combined; a fused gate is the product of its members' matrices.  The
benchmark-circuit table (Sec. 3.1) prints the gate count and depth of each
30-qubit circuit before and after this fusion (QFT: 480 gates at depth 60,
450 gates at depth 58 after fusion).

Reading of the rule (the paper gives it in one sentence): a gate joins the
most recent block among the current last blocks of its qubits when the union
of qubits stays within ``kmax``; otherwise it opens a new block.  Only blocks
that end a qubit's history are candidates, so the merged gate commutes with
every block placed after the one it joins.  No other reordering is done.
"""
import numpy as np

from . import gates as _gates
from . import statevec as _sv


def qubits_of(g):
    return list(g["targets"]) + list(g.get("controls", []))


def greedy_blocks(circuit, kmax=2):
    """List of blocks, each a list of gate indices in application order."""
    blocks = []          # list of [set_of_qubits, [gate indices]]
    last = {}            # qubit -> index of the block that last touched it
    for gi, g in enumerate(circuit):
        qs = qubits_of(g)
        cand = max((last[q] for q in qs if q in last), default=None)
        if cand is not None and len(blocks[cand][0] | set(qs)) <= kmax:
            b = cand
            blocks[b][0].update(qs)
            blocks[b][1].append(gi)
        else:
            b = len(blocks)
            blocks.append([set(qs), [gi]])
        for q in blocks[b][0]:
            # every qubit of the grown block now ends at it (a qubit that only
            # got added here had no later block, so this keeps order valid)
            if last.get(q, -1) <= b:
                last[q] = b
    return [list(m) for _, m in blocks]


def depth(qubit_lists):
    """ASAP layering on qubit occupancy: depth of a sequence of qubit sets."""
    level = {}
    d = 0
    for qs in qubit_lists:
        lv = 1 + max((level.get(q, 0) for q in qs), default=0)
        for q in qs:
            level[q] = lv
        d = max(d, lv)
    return d


def block_qubits(circuit, members):
    qs = set()
    for gi in members:
        qs.update(qubits_of(circuit[gi]))
    return sorted(qs, reverse=True)


def fused_matrix(circuit, members):
    """Product of the member gates embedded in the block's 2^k space.

    Block qubits are listed in decreasing order, so block qubit list[j] is the
    (k-1-j)-th bit of the fused matrix's index; each member is embedded with
    the Kronecker checker and the product taken in application order.
    """
    qs = block_qubits(circuit, members)
    k = len(qs)
    pos = {q: k - 1 - j for j, q in enumerate(qs)}
    M = np.eye(1 << k, dtype=np.complex128)
    for gi in members:
        g = circuit[gi]
        U = _sv.kron_operator(k, _gates.target_matrix(g), [pos[q] for q in g["targets"]],
                              [pos[q] for q in g.get("controls", [])])
        M = U @ M
    return qs, M


def fused_circuit(circuit, kmax=2):
    """The fused circuit as UNITARY gate dicts (targets = block qubits, decreasing)."""
    out = []
    for members in greedy_blocks(circuit, kmax):
        qs, M = fused_matrix(circuit, members)
        out.append({"name": "UNITARY", "targets": qs, "controls": [], "matrix": M})
    return out
