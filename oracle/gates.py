"""Oracle gate matrices (complex128), from their textbook definitions.

Test infrastructure only (see ``oracle/__init__.py``).

The paper names the gates its custom operators specialise (Pauli X, Y, Z and
SWAP in the methodology section, controlled gates, the quantum Fourier
transform of the benchmark-circuit table) but never writes their matrices.
The matrices below follow the standard definitions; the conventions that
change amplitudes (global phases, the fSim sign) are listed in the design
notes under "readings of the paper":

* RX, RY, RZ are exp(-i theta P / 2) for P = X, Y, Z;
* U1(phi) = diag(1, e^{i phi}) (distinct from RZ by a global phase);
* fSim(theta, phi) follows the Foxen et al. (2020) convention;
* sqrt(P) for P in {X, Y, W}, W = (X + Y)/sqrt(2), is the principal square
  root (1+i)/2 I + (1-i)/2 P.

Only the target block is returned: controls are applied by the Eq. 1 loop,
which leaves every amplitude whose control bits are not all 1 unchanged.
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
W = (X + Y) / np.sqrt(2.0)


def _sqrt_pauli(p):
    return 0.5 * (1 + 1j) * I2 + 0.5 * (1 - 1j) * p


def rx(theta):
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta):
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta):
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)


def u1(phi):
    return np.diag([1.0, np.exp(1j * phi)]).astype(np.complex128)


def swap():
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = m[3, 3] = 1.0
    m[1, 2] = m[2, 1] = 1.0
    return m


def fsim(theta, phi):
    c, s = np.cos(theta), np.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = m[2, 2] = c
    m[1, 2] = m[2, 1] = -1j * s
    m[3, 3] = np.exp(-1j * phi)
    return m


# name -> (number of targets, builder(params) -> target block)
_TABLE = {
    "H": (1, lambda p: H.copy()),
    "X": (1, lambda p: X.copy()),
    "Y": (1, lambda p: Y.copy()),
    "Z": (1, lambda p: Z.copy()),
    "SX": (1, lambda p: _sqrt_pauli(X)),
    "SY": (1, lambda p: _sqrt_pauli(Y)),
    "SW": (1, lambda p: _sqrt_pauli(W)),
    "RX": (1, lambda p: rx(p[0])),
    "RY": (1, lambda p: ry(p[0])),
    "RZ": (1, lambda p: rz(p[0])),
    "U1": (1, lambda p: u1(p[0])),
    # controlled forms: the target block is the one-qubit gate, the control
    # comes from the gate's control list
    "CNOT": (1, lambda p: X.copy()),
    "CZ": (1, lambda p: Z.copy()),
    "CU1": (1, lambda p: u1(p[0])),
    "SWAP": (2, lambda p: swap()),
    "FSIM": (2, lambda p: fsim(p[0], p[1])),
}


def target_matrix(gate):
    """Target block of a gate dict ``{"name", "targets", "controls", "params"[, "matrix"]}``."""
    name = gate["name"]
    if name == "UNITARY":
        return np.asarray(gate["matrix"], dtype=np.complex128)
    if name == "DIAG":
        return np.diag(np.asarray(gate["diag"], dtype=np.complex128))
    k, builder = _TABLE[name]
    m = builder(list(gate.get("params", [])))
    assert m.shape == (1 << k, 1 << k)
    return m


def generator(gate):
    """Pauli generator P of a rotation exp(-i theta P / 2), or None."""
    return {"RX": X, "RY": Y, "RZ": Z}.get(gate["name"])
