"""Entangling-gate decomposition (Section 4).  Test infrastructure only.

Eq. (2):  CZ_{i,j} = 1/2 sum_{s=+-1} exp(i (sigma^z_i + sigma^z_j)(x s - pi/4))
with x any solution of cos(2x) = i.  Because sigma^z_i and sigma^z_j commute,
each term is a product of two single-qubit diagonals
D(s) = diag(e^{i(xs - pi/4)}, e^{-i(xs - pi/4)})   (sigma^z |0> = +|0>).

Partitioning the qubits and decomposing every CZ whose qubits lie in
different parts turns the circuit into a sum over branches s in {-1, 1}^S of
tensor products of per-part subcircuits W_p(s), and Eq. (3) gives each
requested coefficient as  <z|C|0> = sum_s prod_p <z_p| W_p(s) |0_p>.

A CNOT whose qubits lie in different parts is the CZ between them with a
Hadamard on its target before and after (H X H = Z), so it is decomposed as
that CZ; the GHZ circuit of Sections 3 and 4 consists of such CNOTs.

Readings taken where the paper is silent:
* branch index b in [0, 2^S): bit k of b selects s_k for the k-th crossing
  gate (CZ or CNOT) in circuit order, bit value 0 -> s_k = +1, 1 -> s_k = -1;
* the factor 1/2 of every decomposed CZ is applied once, as 2^-S, in the sum;
* D(s_k) is applied to both qubits of the k-th crossing CZ at that CZ's
  position in the circuit; for a crossing CNOT(c, t) the target's part
  applies H, D(s_k), H on t at that position and the control's part D(s_k)
  on c;
* inside a part, qubits keep their relative order (local index = rank of the
  qubit among the part's qubits), and z_p collects z's bits in that order.
"""
import math

import numpy as np

from . import gates as G
from . import statevector as sv

# x = pi/4 - (i/2) asinh(1):  cos(2x) = cos(pi/2 - i asinh 1) = sin(i asinh 1) = i sinh(asinh 1) = i
ROOT_X = complex(math.pi / 4.0, -0.5 * math.asinh(1.0))
ROOTS = (ROOT_X, -ROOT_X, ROOT_X + math.pi)


def branch_diag(s: int, x: complex = ROOT_X) -> np.ndarray:
    """Single-qubit factor of one term of Eq. (2): exp(i sigma^z (x s - pi/4))."""
    a = 1j * (x * s - math.pi / 4.0)
    return np.diag([np.exp(a), np.exp(-a)]).astype(np.complex128)


def eq2_sum(x: complex = ROOT_X) -> np.ndarray:
    """Right-hand side of Eq. (2) as a 4x4 matrix (index b_i + 2 b_j)."""
    total = np.zeros((4, 4), dtype=np.complex128)
    for s in (1, -1):
        d = branch_diag(s, x)
        total += np.kron(d, d)   # kron(A_j, A_i): both diagonal, order irrelevant
    return 0.5 * total


def crossing_gates(circuit, part) -> list:
    """Positions of the decomposed gates (CZ or CNOT with qubits in different
    parts), in circuit order.  A controlled phase across parts is rejected."""
    pos = []
    for k, rec in enumerate(circuit):
        op = int(rec["op"])
        if op in (G.OP_CNOT, G.OP_CZ, G.OP_CP):
            a, b = int(rec["q0"]), int(rec["q1"])
            if part[a] != part[b]:
                if op == G.OP_CP:
                    raise ValueError("only CZ and CNOT gates may cross partitions")
                pos.append(k)
    return pos


def _local_maps(part, nparts):
    qubits = [[q for q in range(len(part)) if part[q] == p] for p in range(nparts)]
    local = {}
    for p in range(nparts):
        for r, q in enumerate(qubits[p]):
            local[q] = r
    return qubits, local


def subcircuit_states(n: int, circuit, part, branch: int, x: complex = ROOT_X):
    """W_p(s) |0_p> for every part p, s given by the bits of ``branch``."""
    part = np.asarray(part)
    nparts = int(part.max()) + 1
    qubits, local = _local_maps(part, nparts)
    states = [sv.init_state(len(qubits[p])) for p in range(nparts)]
    k = 0
    for rec in circuit:
        op = int(rec["op"])
        a = int(rec["q0"])
        if op in (G.OP_CNOT, G.OP_CZ, G.OP_CP):
            b = int(rec["q1"])
            if part[a] != part[b]:
                s = 1 if ((branch >> k) & 1) == 0 else -1
                d = branch_diag(s, x)
                pb = part[b]
                if op == G.OP_CNOT:  # target b: H before the CZ's factor
                    sv.apply_1q(states[pb], len(qubits[pb]), local[b], G.H)
                for q in (a, b):
                    p = part[q]
                    sv.apply_1q(states[p], len(qubits[p]), local[q], d)
                if op == G.OP_CNOT:  # and after it
                    sv.apply_1q(states[pb], len(qubits[pb]), local[b], G.H)
                k += 1
                continue
            p = part[a]
            loc = rec.copy()
            loc["q0"], loc["q1"] = local[a], local[b]
            sv.apply_record(states[p], len(qubits[p]), loc)
        else:
            p = part[a]
            loc = rec.copy()
            loc["q0"] = local[a]
            sv.apply_record(states[p], len(qubits[p]), loc)
    return states, qubits


def split_bitstring(z: int, qubits_p) -> int:
    """z_p: the bits of z at the part's qubits, in ascending qubit order."""
    out = 0
    for r, q in enumerate(qubits_p):
        out |= ((z >> q) & 1) << r
    return out


def branch_amplitudes(n: int, circuit, part, zs, x: complex = ROOT_X) -> np.ndarray:
    """Eq. (3): <z|C|0> = 2^-S sum_b prod_p <z_p|W_p(s_b)|0_p> for every z in
    ``zs``, summed over all 2^S branches with math.fsum on real and imaginary
    parts separately."""
    zs = [int(z) for z in zs]
    S = len(crossing_gates(circuit, part))
    terms = np.empty((1 << S, len(zs)), dtype=np.complex128)
    for b in range(1 << S):
        states, qubits = subcircuit_states(n, circuit, part, b, x)
        for m, z in enumerate(zs):
            prod = 1.0 + 0.0j
            for p, st in enumerate(states):
                prod *= st[split_bitstring(z, qubits[p])]
            terms[b, m] = prod
    scale = 2.0 ** (-S)
    return np.array([complex(math.fsum(terms[:, m].real) * scale,
                             math.fsum(terms[:, m].imag) * scale) for m in range(len(zs))])


def projector_amplitudes(n: int, circuit, part, zs) -> np.ndarray:
    """Independent second branch sum: CZ_{i,j} = |0><0|_i (x) I_j + |1><1|_i (x) Z_j
    and CNOT_{c,t} = |0><0|_c (x) I_t + |1><1|_c (x) X_t (no Hadamards).
    Branch bit 0 -> (|0><0| on the first qubit, I on the second), bit 1 ->
    (|1><1| on the first, Z or X on the second).  No prefactor.  Must agree
    with ``branch_amplitudes``."""
    part = np.asarray(part)
    nparts = int(part.max()) + 1
    qubits, local = _local_maps(part, nparts)
    zs = [int(z) for z in zs]
    S = len(crossing_gates(circuit, part))
    p0 = np.diag([1.0, 0.0]).astype(np.complex128)
    p1 = np.diag([0.0, 1.0]).astype(np.complex128)
    terms = np.empty((1 << S, len(zs)), dtype=np.complex128)
    for br in range(1 << S):
        states = [sv.init_state(len(qubits[p])) for p in range(nparts)]
        k = 0
        for rec in circuit:
            op = int(rec["op"])
            a = int(rec["q0"])
            two = op in (G.OP_CNOT, G.OP_CZ, G.OP_CP)
            if two and part[a] != part[int(rec["q1"])]:
                b = int(rec["q1"])
                bit = (br >> k) & 1
                pa, pb = part[a], part[b]
                sv.apply_1q(states[pa], len(qubits[pa]), local[a], p1 if bit else p0)
                if bit:
                    sv.apply_1q(states[pb], len(qubits[pb]), local[b], G.X if op == G.OP_CNOT else G.Z)
                k += 1
                continue
            p = part[a]
            loc = rec.copy()
            loc["q0"] = local[a]
            if two:
                loc["q1"] = local[int(rec["q1"])]
            sv.apply_record(states[p], len(qubits[p]), loc)
        for m, z in enumerate(zs):
            prod = 1.0 + 0.0j
            for p, st in enumerate(states):
                prod *= st[split_bitstring(z, qubits[p])]
            terms[br, m] = prod
    return np.array([complex(math.fsum(terms[:, m].real), math.fsum(terms[:, m].imag))
                     for m in range(len(zs))])
