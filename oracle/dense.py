"""Brute-force dense 2^n x 2^n gate matrices (n <= 10).  Test infrastructure
only (see package doc).

Section 2: gate operations on N qubits are matrix-vector products with
2^N x 2^N unitary matrices.  Each k-qubit gate g (2^k x 2^k) is embedded
entry by entry:  M[i, j] = g[sub(i), sub(j)] if i and j agree on every
non-target bit, else 0, with sub(i) = sum_j b_{targets[j]}(i) 2^j.  This is
independent of the pair loops in ``statevector`` and pins them.
"""
import numpy as np

from . import gates as G

MAX_DENSE_QUBITS = 10


def embed(n: int, targets, g: np.ndarray) -> np.ndarray:
    if n > MAX_DENSE_QUBITS:
        raise ValueError("dense embedding limited to n <= 10")
    targets = list(targets)
    dim = 1 << n
    idx = np.arange(dim)
    sub = np.zeros(dim, dtype=np.int64)
    tmask = 0
    for j, q in enumerate(targets):
        sub |= ((idx >> q) & 1) << j
        tmask |= 1 << q
    rest = idx & ~tmask
    same_rest = rest[:, None] == rest[None, :]
    return np.where(same_rest, g[sub[:, None], sub[None, :]], 0.0).astype(np.complex128)


def circuit_matrix(n: int, circuit) -> np.ndarray:
    """Product G_L ... G_1 of the dense embeddings of every gate record."""
    m = np.eye(1 << n, dtype=np.complex128)
    for rec in circuit:
        qubits, g = G.record_matrix(rec)
        m = embed(n, qubits, g) @ m
    return m


def run_dense(n: int, circuit, basis_index: int = 0) -> np.ndarray:
    e = np.zeros(1 << n, dtype=np.complex128)
    e[basis_index] = 1.0
    for rec in circuit:
        qubits, g = G.record_matrix(rec)
        e = embed(n, qubits, g) @ e
    return e
