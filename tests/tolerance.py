"""Complex64 rounding bound of a circuit.

Amplitudes of a normalised complex64 state must agree with the complex128
oracle within 1e-5 (max-abs).  Tests of long circuits also hold the 2-norm
of the whole error vector to the first-order worst-case bound of FP32
rounding, which grows with the gate count.  The bound, with u = 2^-24 and
every gate unitary (so an error already made is carried, not amplified, by
later gates):

* input: the state is rounded to complex64 once: u;
* a dense gate on k targets (m = 2^k, matrix rounded to FP32) changes each
  output by at most (sqrt(2) (m + 1) + 1) u (|G| |psi|)_i: m complex
  products and m - 1 additions in FP32, plus the matrix rounding.  With
  ||  |G|  ||_2 <= ||G||_F = sqrt(m) and one rounding of the stored result,
  the 2-norm of the error is at most e(k) u, e(k) = (sqrt(2) (m + 1) + 1)
  sqrt(m) + 1: e(1) = 8.4, e(2) = 17.1, e(3) = 40.9, e(6) = 744;
* a diagonal gate (Z, RZ, U1, CZ, CU1, DIAG): one complex product, the
  rounded factor and the stored result: 4 u;
* X, Y, SWAP, CNOT move amplitudes (Y with factors +-i): exact.

Controls restrict a gate to a subspace and do not add to its error.  A plan
that fuses gates into blocks of up to w qubits applies each block as one
dense gate; there are at most as many blocks as gates, so every gate is
counted with max(k, w) targets.
"""
import math

U32 = 2.0 ** -24

MOVES = {"X", "Y", "SWAP", "CNOT"}
DIAGONAL = {"Z", "RZ", "U1", "CZ", "CU1", "DIAG"}


def dense_error(k):
    """e(k): worst-case 2-norm error of one dense k-target gate, in units of u."""
    m = 2 ** k
    return (math.sqrt(2.0) * (m + 1) + 1.0) * math.sqrt(m) + 1.0


def c64_bound(gates, width=1):
    """First-order worst-case 2-norm of the FP32 rounding error of a circuit."""
    total = 1.0
    for g in gates:
        k = max(len(g["targets"]), width)
        if width <= 1 and g["name"] in MOVES:
            continue
        if width <= 1 and g["name"] in DIAGONAL:
            total += 4.0
            continue
        total += dense_error(k)
    return total * U32

