"""FP64 state-vector simulator.  Test infrastructure only (see package doc).

The state of n qubits is a vector of 2^n complex numbers (Section 2); qubit q
is bit q of the amplitude index.  Every gate is applied in place, one pass
over the vector, exactly as the definitions below state; nothing is fused or
reordered.
"""
import math

import numpy as np

from . import gates as G

_CHUNK = 1 << 22  # amplitudes per temporary, to bound host memory at large n


def init_state(n: int, basis_index: int = 0) -> np.ndarray:
    """|basis_index>; the computer starts in |0...0> (Section 4, before Eq. (3))."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[basis_index] = 1.0
    return psi


def _pair_update(v: np.ndarray, axis: int, u: np.ndarray) -> None:
    """Eq. (1) on every pair along ``axis`` (length 2) of the view ``v``:
    (a0, a1) <- U (a0, a1), with a0 at index 0 of that axis."""
    _pairs(np.moveaxis(v, axis, 0), u)      # a view: writes reach psi


def _pairs(v: np.ndarray, u: np.ndarray) -> None:
    # v has shape (2, ...); split the remaining axes until a piece is small
    size = v[0].size
    if size <= _CHUNK:
        a0 = v[0].copy()
        a1 = v[1].copy()
        v[0] = u[0, 0] * a0 + u[0, 1] * a1
        v[1] = u[1, 0] * a0 + u[1, 1] * a1
        return
    d1 = v.shape[1]
    if v.ndim == 2:
        for s in range(0, d1, _CHUNK):
            _pairs(v[:, s:s + _CHUNK], u)
        return
    step = (d1 * _CHUNK) // size
    if step >= 1:
        for s in range(0, d1, step):
            _pairs(v[:, s:s + step], u)
    else:
        for s in range(d1):
            _pairs(v[:, s], u)


def apply_1q(psi: np.ndarray, n: int, t: int, u: np.ndarray) -> None:
    """Eq. (1): for every index i with bit t = 0 and j = i + 2^t,
    (psi_i, psi_j) <- U (psi_i, psi_j)."""
    v = psi.reshape(1 << (n - 1 - t), 2, 1 << t)
    _pair_update(v, 1, u)


def apply_controlled(psi: np.ndarray, n: int, c: int, t: int, u: np.ndarray) -> None:
    """Controlled-U: Eq. (1) on target t restricted to indices whose control
    bit c is 1 (CNOT = controlled-X, CZ = controlled-Z, CP = controlled
    diag(1, e^{i theta}); Sections 3 and 4)."""
    if c == t:
        raise ValueError("control equals target")
    hi, lo = max(c, t), min(c, t)
    v = psi.reshape(1 << (n - 1 - hi), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    if c == hi:
        sub = v[:, 1]          # (A, M, 2, L): target axis 2
        _pair_update(sub, 2, u)
    else:
        sub = v[:, :, :, 1]    # (A, 2, M, L): target axis 1
        _pair_update(sub, 1, u)


def apply_matrix(psi: np.ndarray, n: int, targets, m: np.ndarray) -> None:
    """psi <- (M on ``targets``) psi for a dense 2^k x 2^k matrix M whose
    row/column index is r = sum_j b_{targets[j]} 2^j: the 2^n x 2^n
    embedding of a k-qubit gate (Section 2), computed as a tensor contraction
    over the target axes."""
    targets = list(targets)
    k = len(targets)
    if len(set(targets)) != k:
        raise ValueError("targets must be distinct")
    t = psi.reshape([2] * n)                  # axis a <-> qubit n-1-a
    axes = [n - 1 - q for q in reversed(targets)]  # targets[k-1] first (high bit of r)
    moved = np.moveaxis(t, axes, list(range(k)))
    shape = moved.shape
    res = m @ moved.reshape(1 << k, -1)
    res = np.moveaxis(res.reshape(shape), list(range(k)), axes)
    psi[:] = res.reshape(-1)


def apply_record(psi: np.ndarray, n: int, rec) -> None:
    op = int(rec["op"])
    if op in G.NAMED_1Q:
        apply_1q(psi, n, int(rec["q0"]), G.NAMED_1Q[op])
    elif op == G.OP_U:
        apply_1q(psi, n, int(rec["q0"]), G.u_from_record(rec["u"]))
    elif op == G.OP_CNOT:
        apply_controlled(psi, n, int(rec["q0"]), int(rec["q1"]), G.X)
    elif op == G.OP_CZ:
        apply_controlled(psi, n, int(rec["q0"]), int(rec["q1"]), G.Z)
    elif op == G.OP_CP:
        apply_controlled(psi, n, int(rec["q0"]), int(rec["q1"]), G.phase(float(rec["theta"])))
    else:
        raise ValueError(f"unknown op {op}")


def run_circuit(n: int, circuit, psi: np.ndarray | None = None, basis_index: int = 0) -> np.ndarray:
    """psi_out = G_L ... G_1 |basis_index>, one gate at a time in circuit order."""
    if psi is None:
        psi = init_state(n, basis_index)
    for rec in circuit:
        apply_record(psi, n, rec)
    return psi


def norm(psi: np.ndarray) -> float:
    """sum_i |psi_i|^2 in FP64 (the normalisation of Section 2), chunk sums
    combined with math.fsum so the result does not depend on chunking."""
    parts = []
    for a in range(0, psi.size, _CHUNK):
        c = psi[a:a + _CHUNK]
        parts.append(float(np.sum(c.real * c.real + c.imag * c.imag)))
    return math.fsum(parts)


def amplitudes(psi: np.ndarray, idx) -> np.ndarray:
    """Coefficients <z|psi> for the requested basis indices z (Section 4)."""
    return psi[np.asarray(idx, dtype=np.int64)]


def permute_qubits(psi: np.ndarray, n: int, perm) -> np.ndarray:
    """Relabel qubits: the returned state has bit perm[q] equal to bit q of
    the input index, i.e. out[sum_q b_q 2^perm[q]] = psi[sum_q b_q 2^q]."""
    perm = list(perm)
    idx = np.arange(1 << n, dtype=np.int64)
    dst = np.zeros_like(idx)
    for q in range(n):
        dst |= ((idx >> q) & 1) << perm[q]
    out = np.empty_like(psi)
    out[dst] = psi
    return out
