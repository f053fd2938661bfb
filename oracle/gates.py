"""Textbook gate matrices (FP64).  Test infrastructure only (see package doc).

Single-qubit gates act as in Eq. (1) of Section 2: (a0, a1) <- U (a0, a1),
where a0 is the amplitude with the target bit 0.  Two-qubit matrices use the
row/column index r = b_first + 2*b_second.
"""
import numpy as np

# op codes of the gate records (same numbering as the record producer)
OP_H, OP_X, OP_Y, OP_Z, OP_S, OP_T, OP_U, OP_CNOT, OP_CZ, OP_CP = range(10)

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, np.exp(0.25j * np.pi)]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)

NAMED_1Q = {OP_H: H, OP_X: X, OP_Y: Y, OP_Z: Z, OP_S: S, OP_T: T}


def u_from_record(u8) -> np.ndarray:
    """2x2 matrix stored row-major as (re, im) pairs."""
    u8 = np.asarray(u8, dtype=np.float64).reshape(2, 2, 2)
    return u8[..., 0] + 1j * u8[..., 1]


def phase(theta: float) -> np.ndarray:
    """diag(1, e^{i theta}): the single-qubit part of controlled-phase."""
    return np.array([[1, 0], [0, np.exp(1j * theta)]], dtype=np.complex128)


def controlled(u: np.ndarray) -> np.ndarray:
    """4x4 controlled-U with the control as the first qubit (index bit 0) and
    the target as the second (index bit 1): U acts where the control is 1."""
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = m[2, 2] = 1.0          # control = 0: identity on the target
    m[1, 1], m[1, 3] = u[0, 0], u[0, 1]
    m[3, 1], m[3, 3] = u[1, 0], u[1, 1]
    return m


def record_matrix(rec) -> tuple:
    """(qubits, matrix) of one gate record, matrix in the index convention
    r = sum_j b_{qubits[j]} 2^j."""
    op = int(rec["op"])
    if op in NAMED_1Q:
        return (int(rec["q0"]),), NAMED_1Q[op]
    if op == OP_U:
        return (int(rec["q0"]),), u_from_record(rec["u"])
    if op == OP_CNOT:
        return (int(rec["q0"]), int(rec["q1"])), controlled(X)
    if op == OP_CZ:
        return (int(rec["q0"]), int(rec["q1"])), np.diag([1, 1, 1, -1]).astype(np.complex128)
    if op == OP_CP:
        return (int(rec["q0"]), int(rec["q1"])), np.diag([1, 1, 1, np.exp(1j * float(rec["theta"]))])
    raise ValueError(f"unknown op {op}")
