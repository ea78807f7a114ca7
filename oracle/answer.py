"""Answer-string estimation from the full distribution (test infrastructure).

Sec. "Estimating the answer string": the qubits are fixed one after another;
for qubit k the probability of reading 0 together with the values already
chosen for qubits 0..k-1 is set against that of reading 1, the likelier
value is kept, and equally likely values (within a relative tolerance) take
a given random draw. Here each of those probabilities is read off the FP64
distribution |psi_x|^2 by summing out the qubits not yet fixed.
"""
import numpy as np


def answer_string(psi, tie_tol, tie_draws):
    """psi: state vector as an array of shape (2,)*n (qubit 0 = axis 0).
    Returns (bits, probs) as the GPU routine does."""
    n = psi.ndim
    rest = np.abs(psi) ** 2           # distribution restricted to the chosen prefix
    p_prefix = float(rest.sum())
    bits, probs = [], []
    for k in range(n):
        p0 = float(rest[0].sum())
        p1 = float(rest[1].sum())
        if abs(p0 - p1) <= tie_tol * p_prefix:
            b = int(tie_draws[k])
        else:
            b = 0 if p0 > p1 else 1
        bits.append(b)
        probs.append((p0, p1))
        p_prefix = p0 if b == 0 else p1
        rest = rest[b]
    return bits, probs
