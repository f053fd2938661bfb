"""Single-qubit expectation values (Section 3).  Test infrastructure only.

<Q_alpha(i)> = (1 - <psi| sigma^alpha_i |psi>) / 2 for alpha = x, y, z,
computed from the definition: apply the Pauli matrix to a copy of the state
and take the inner product.  For the uniform superposition H^{(x)N}|0> the
exact values are 0 (x) and 1/2 (y, z).
"""
import numpy as np

from . import gates as G
from . import statevector as sv

PAULI = {"x": G.X, "y": G.Y, "z": G.Z}


def pauli_expectation(psi: np.ndarray, n: int, q: int, alpha: str) -> float:
    phi = psi.copy()
    sv.apply_1q(phi, n, q, PAULI[alpha])
    return float(np.vdot(psi, phi).real)


def q_expectations(psi: np.ndarray, n: int) -> np.ndarray:
    """Array of shape (n, 3): <Q_x(i)>, <Q_y(i)>, <Q_z(i)> for every qubit."""
    out = np.empty((n, 3))
    for q in range(n):
        for a, alpha in enumerate("xyz"):
            out[q, a] = 0.5 * (1.0 - pauli_expectation(psi, n, q, alpha))
    return out
