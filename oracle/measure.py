"""Oracle measurement operators.  Test infrastructure only.

The methodology section (Sec. 2) lists, besides the gate operators, an
operator that collapses a state onto a measurement outcome and re-normalises
it, and shot frequencies sampled with the Metropolis algorithm (Metropolis et
al. 1953).  The paper gives no formulas; the readings used here:

* outcome index m of measured qubits q_0..q_{r-1}: m = sum_j bit(q_j) 2^(r-1-j)
  (q_0 is the most significant bit), as for the probabilities;
* collapse: psi' = P_m psi / ||P_m psi|| with P_m the projector onto the
  basis states whose measured bits spell m; when ||P_m psi|| = 0 every
  amplitude becomes 0;
* inverse-CDF sampling: with c_m = p_0 + ... + p_m (summed in index order)
  and T = c_{R-1}, a uniform u in [0, 1) gives the smallest m with
  u T < c_m; when the product u T rounds up to T, the last outcome of
  non-zero probability;
* Metropolis frequencies: independent chains; chain c starts at outcome
  x = start_c and at each step s takes the proposal y = y_{s,c} when
  u_{s,c} p(x) < p(y) (acceptance probability min(1, p(y)/p(x)), a proposal
  drawn uniformly is symmetric), then counts the outcome x it holds.  Every
  random number is an input.
"""
import numpy as np


def outcome_index(i, qubits):
    """Outcome index of basis state i for the measured qubits (qubits[0] = MSB)."""
    r = len(qubits)
    return sum(((int(i) >> q) & 1) << (r - 1 - j) for j, q in enumerate(qubits))


def projector_mask(n, qubits, m):
    """Boolean mask over the 2^n basis states of the range of P_m."""
    idx = np.arange(1 << n, dtype=np.int64)
    r = len(qubits)
    keep = np.ones(1 << n, dtype=bool)
    for j, q in enumerate(qubits):
        keep &= ((idx >> q) & 1) == ((m >> (r - 1 - j)) & 1)
    return keep


def collapse(state, qubits, m):
    """P_m psi / ||P_m psi|| (complex128) and ||P_m psi||^2 (methodology
    section: collapse and re-normalisation)."""
    psi = np.asarray(state, dtype=np.complex128)
    n = int(psi.size).bit_length() - 1
    out = np.where(projector_mask(n, qubits, m), psi, 0.0)
    p = float(np.sum(out.real ** 2 + out.imag ** 2))
    if p == 0.0:
        return np.zeros_like(out), 0.0
    return out / np.sqrt(p), p


def cumulative(probs):
    """c_m = p_0 + ... + p_m, summed one term at a time in index order."""
    p = np.asarray(probs, dtype=np.float64)
    c = np.empty_like(p)
    s = 0.0
    for m in range(p.size):
        s += p[m]
        c[m] = s
    return c


def sample_inverse_cdf(probs, uniforms):
    """Smallest m with u T < c_m for every uniform u (T = c_{R-1}); a binary
    search of the sorted c (numpy's searchsorted); the last outcome of
    non-zero probability when u T rounds up to T."""
    p = np.asarray(probs, dtype=np.float64)
    c = cumulative(p)
    x = np.asarray(uniforms, dtype=np.float64) * c[-1]
    m = np.searchsorted(c, x, side="right")
    nz = np.nonzero(p)[0]
    last = int(nz[-1]) if nz.size else 0
    return np.where(m >= c.size, last, m).astype(np.int64)


def metropolis_counts(probs, starts, proposals, uniforms):
    """Frequencies of independent Metropolis chains.

    ``starts`` [C]; ``proposals`` and ``uniforms`` [steps, C].  Returns counts
    [R] (int64) of the outcome each chain holds after each step."""
    p = np.asarray(probs, dtype=np.float64)
    prop = np.asarray(proposals, dtype=np.int64)
    uni = np.asarray(uniforms, dtype=np.float64)
    counts = np.zeros(p.size, dtype=np.int64)
    steps, C = prop.shape
    for c in range(C):
        x = int(starts[c])
        for s in range(steps):
            y = int(prop[s, c])
            if uni[s, c] * p[x] < p[y]:
                x = y
            counts[x] += 1
    return counts
