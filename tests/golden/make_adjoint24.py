"""Write ``adjoint24_cfg4.txt``: oracle gradients of the 24-qubit
hardware-efficient ansatz (12 layers of RY, RZ on every qubit and a CZ ring,
576 angles uniform in [0, 2 pi), seed 0) for the energy of
H = sum Z_i Z_{i+1} + 0.5 sum X_i (open chain), starting from |0..0>.

Calls only ``oracle/`` (and the seeded generators in ``workloads/``):

* the oracle's adjoint gradient of every angle (oracle.adjoint.grad_adjoint);
* parameter shift, [E(t + pi/2) - E(t - pi/2)] / 2, and central finite
  differences with step 1e-5, on a seeded subset of 32 angles.

E(t +- s) is the same computation as oracle.adjoint.expval on the shifted
circuit: the gates before the shifted one are applied once and their
output reused for every shift of that angle (the same gate applications in
the same order, so the same numbers), which halves the run time.  Takes
about an hour on 8 cores.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint as OA  # noqa: E402
from oracle import statevec as S  # noqa: E402

N, LAYERS, SEED, SUBSET, STEP = 24, 12, 0, 32, 1e-5
OUT = os.path.join(HERE, "adjoint24_cfg4.txt")


def shifted_energies(circ, gi, psi_before, shifts):
    """E with the angle of gate gi moved by each shift; psi_before is the state
    in front of gate gi."""
    out = []
    a = np.empty_like(psi_before)
    b = np.empty_like(psi_before)
    for sh in shifts:
        g = dict(circ[gi])
        g["params"] = [g["params"][0] + sh] + list(g["params"][1:])
        S.apply_gate(psi_before, g, out=a)
        for g2 in circ[gi + 1:]:
            S.apply_gate(a, g2, out=b)
            a, b = b, a
        out.append(S.expval_tfim(a, 1.0, 0.5, False))
    return out


def main():
    circ = W.variational(N, LAYERS, seed=SEED)
    slots = W.parameter_slots(circ)
    rng = np.random.default_rng(SEED)
    subset = sorted(int(i) for i in rng.choice(len(slots), size=SUBSET, replace=False))
    t0 = time.time()
    energy, adj = OA.grad_adjoint(circ, N)
    print("adjoint done in %.0f s, E = %.12f" % (time.time() - t0, energy), flush=True)
    ps, fd = {}, {}
    psi = S.basis_state(N, 0)
    tmp = np.empty_like(psi)
    pos = 0
    for p in subset:
        gi = slots[p]
        while pos < gi:   # advance the shared prefix to the front of gate gi
            S.apply_gate(psi, circ[pos], out=tmp)
            psi, tmp = tmp, psi
            pos += 1
        e = shifted_energies(circ, gi, psi, [math.pi / 2, -math.pi / 2, STEP, -STEP])
        ps[p] = 0.5 * (e[0] - e[1])
        fd[p] = (e[2] - e[3]) / (2 * STEP)
        print("param %d (gate %d): ps %.12e fd %.12e adjoint %.12e  %.0f s" % (
            p, gi, ps[p], fd[p], adj[p], time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle gradients of <H>, H = sum Z_i Z_{i+1} + 0.5 sum X_i (open chain), for the\n")
        f.write("# %d-qubit hardware-efficient ansatz (%d layers RY, RZ, CZ ring; angles U[0, 2pi) seed %d)\n"
                % (N, LAYERS, SEED))
        f.write("# from |0..0>.  Written by tests/golden/make_adjoint24.py, which calls only oracle/.\n")
        f.write("# energy %.17e\n" % energy)
        f.write("# adjoint: index gradient (every angle, circuit order)\n")
        f.write("# subset: index parameter_shift finite_difference(step %g)\n" % STEP)
        for i, g in enumerate(adj):
            f.write("adjoint %d %.17e\n" % (i, g))
        for p in subset:
            f.write("subset %d %.17e %.17e\n" % (p, ps[p], fd[p]))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
