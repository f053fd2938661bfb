"""Seeded synthetic workloads: circuits (gate records) and bitstrings.

This module only draws random numbers and lays out gate records.  It holds
none of the simulation arithmetic: both the GPU library and the CPU oracle
read the records it produces and each builds its own gate matrices from the
op codes.  Random data that the method consumes (Haar-random 2x2 unitaries,
controlled-phase angles) is drawn here and handed over inside the records.

Circuit families (the paper's own random circuits follow rules that are not
part of the paper, so layered Haar+CZ circuits of the same structure stand in:
layers of dense single-qubit gates plus CZ patterns, Section 4):

* ``random_mixed``      -- uniform mix of named 1q gates and CNOT/CZ/CP pairs
* ``layered_brick``     -- Haar U(2) on every qubit, CZ on alternating
                           nearest-neighbour bricks
* ``layered_random_pairs`` -- Haar U(2) on every qubit, CZ on a seeded set of
                           disjoint random pairs
* ``grid_circuit``      -- 6x8 grid, Haar layers + CZ on 4 alternating edge
                           patterns, with a 24|24 cut (Section 4, Eq. (3))
* ``ghz`` / ``hadamard_all`` / ``qft`` -- known-outcome circuits (Section 3)

Index convention: qubit q is bit q of the amplitude index (little endian).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Gate record layout.  Must match ``juqcs_gate`` in include/juqcs_gpu.h.
# --------------------------------------------------------------------------
OP_H, OP_X, OP_Y, OP_Z, OP_S, OP_T, OP_U, OP_CNOT, OP_CZ, OP_CP = range(10)
OP_NAMES = ["H", "X", "Y", "Z", "S", "T", "U", "CNOT", "CZ", "CP"]
ONE_QUBIT_OPS = (OP_H, OP_X, OP_Y, OP_Z, OP_S, OP_T, OP_U)
TWO_QUBIT_OPS = (OP_CNOT, OP_CZ, OP_CP)

GATE_DTYPE = np.dtype(
    [
        ("op", "<i4"),      # OP_* code
        ("q0", "<i4"),      # 1q: target.  CNOT: control.  CZ/CP: first qubit
        ("q1", "<i4"),      # CNOT: target.  CZ/CP: second qubit.  1q: -1
        ("pad", "<i4"),
        ("theta", "<f8"),   # CP angle
        ("u", "<f8", (8,)), # OP_U: 2x2 row-major, (re, im) pairs
    ],
    align=True,
)
assert GATE_DTYPE.itemsize == 88


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def empty_circuit(count: int) -> np.ndarray:
    g = np.zeros(count, dtype=GATE_DTYPE)
    g["q1"] = -1
    return g


def gate(op: int, q0: int, q1: int = -1, theta: float = 0.0, u=None) -> np.ndarray:
    g = empty_circuit(1)
    g["op"], g["q0"], g["q1"], g["theta"] = op, q0, q1, theta
    if u is not None:
        m = np.asarray(u, dtype=np.complex128).reshape(2, 2)
        g["u"][0] = np.stack([m.real, m.imag], axis=-1).reshape(8)
    return g


def concat(*parts) -> np.ndarray:
    parts = [p for p in parts if len(p)]
    return np.concatenate(parts) if parts else empty_circuit(0)


def haar_u2(rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed 2x2 unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal folded back into Q (F. Mezzadri, Notices AMS 54,
    2007).  This is random input generation, not a simulation step."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def _u_record(m: np.ndarray) -> np.ndarray:
    return np.stack([m.real, m.imag], axis=-1).reshape(8)


def haar_u2_many(rng: np.random.Generator, count: int) -> np.ndarray:
    """count Haar-distributed 2x2 unitaries at once (same construction as
    haar_u2, stacked QR), returned as (count, 8) gate-record rows."""
    z = (rng.standard_normal((count, 2, 2)) + 1j * rng.standard_normal((count, 2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    u = q * (d / np.abs(d))[:, None, :]
    return np.stack([u.real, u.imag], axis=-1).reshape(count, 8)


# --------------------------------------------------------------------------
# Circuit families
# --------------------------------------------------------------------------
def random_mixed(n: int, count: int, seed: int, p1: float = 0.6) -> np.ndarray:
    """Each gate is single-qubit with probability p1 (type uniform over
    H, X, Y, Z, S, T, Haar U(2); target uniform), otherwise two-qubit (type
    uniform over CNOT, CZ, CP(theta ~ U[0, 2pi)); ordered distinct pair)."""
    rng = _rng(seed)
    g = empty_circuit(count)
    for k in range(count):
        if rng.random() < p1:
            op = int(rng.integers(0, 7))
            g["op"][k] = op
            g["q0"][k] = int(rng.integers(0, n))
            if op == OP_U:
                g["u"][k] = _u_record(haar_u2(rng))
        else:
            op = OP_CNOT + int(rng.integers(0, 3))
            a = int(rng.integers(0, n))
            b = int(rng.integers(0, n - 1))
            if b >= a:
                b += 1
            g["op"][k], g["q0"][k], g["q1"][k] = op, a, b
            if op == OP_CP:
                g["theta"][k] = float(rng.uniform(0.0, 2.0 * np.pi))
    return g


def layered_brick(n: int, layers: int, seed: int) -> np.ndarray:
    """Layer l: Haar U(2) on qubits 0..n-1 in order, then CZ(q, q+1) for every
    q with q = l (mod 2) and q+1 < n."""
    rng = _rng(seed)
    out = []
    for layer in range(layers):
        g = empty_circuit(n)
        g["op"] = OP_U
        g["q0"] = np.arange(n)
        for q in range(n):
            g["u"][q] = _u_record(haar_u2(rng))
        out.append(g)
        qs = [q for q in range(layer % 2, n - 1, 2)]
        cz = empty_circuit(len(qs))
        cz["op"] = OP_CZ
        cz["q0"] = qs
        cz["q1"] = [q + 1 for q in qs]
        out.append(cz)
    return concat(*out)


def layered_random_pairs(n: int, depth: int, rng: np.random.Generator) -> np.ndarray:
    """Layer: Haar U(2) on qubits 0..n-1, then floor(n/2) disjoint CZ pairs
    taken as consecutive elements of a seeded shuffle of the qubits."""
    out = []
    for _ in range(depth):
        g = empty_circuit(n)
        g["op"] = OP_U
        g["q0"] = np.arange(n)
        g["u"] = haar_u2_many(rng, n)
        out.append(g)
        perm = rng.permutation(n)
        npair = n // 2
        cz = empty_circuit(npair)
        cz["op"] = OP_CZ
        cz["q0"] = perm[0 : 2 * npair : 2]
        cz["q1"] = perm[1 : 2 * npair : 2]
        out.append(cz)
    return concat(*out)


def batch_shape(i: int, master_seed: int = 4, nmin: int = 12, nmax: int = 24,
                dmin: int = 10, dmax: int = 40):
    """(n, depth) of batch instance i (the first two draws of its seed)."""
    rng = _rng(master_seed * (1 << 32) + i)
    n = int(rng.integers(nmin, nmax + 1))
    depth = int(rng.integers(dmin, dmax + 1))
    return n, depth


def batch_instance(i: int, master_seed: int = 4, nmin: int = 12, nmax: int = 24,
                   dmin: int = 10, dmax: int = 40):
    """Instance i of batch_instances: seed master*2^32 + i, n ~ U{nmin..nmax},
    depth ~ U{dmin..dmax} (both inclusive), layered_random_pairs."""
    rng = _rng(master_seed * (1 << 32) + i)
    n = int(rng.integers(nmin, nmax + 1))
    depth = int(rng.integers(dmin, dmax + 1))
    return n, layered_random_pairs(n, depth, rng)


def batch_instances(count: int, master_seed: int = 4, nmin: int = 12, nmax: int = 24,
                    dmin: int = 10, dmax: int = 40):
    """Independent circuits; instance i is batch_instance(i)."""
    return [batch_instance(i, master_seed, nmin, nmax, dmin, dmax) for i in range(count)]


def batch_bitstrings(i: int, n: int, count: int = 64) -> np.ndarray:
    """The seeded bitstrings read out of batch instance i (seed 10000 + i)."""
    return bitstrings(n, count, seed=10_000 + i)


def grid_qubit(r: int, c: int, rows: int) -> int:
    """Column-major numbering q = rows*c + r, so the left half of the columns
    holds the low qubits."""
    return rows * c + r


def _grid_pattern_edges(layer: int, rows: int, cols: int):
    """CZ edges of layer ``layer``: pattern "ABCD"[layer mod 4] (A: horizontal
    (r,c)-(r,c+1) with r+c even; B: horizontal, r+c odd; C: vertical
    (r,c)-(r+1,c), r+c even; D: vertical, r+c odd), ordered by ascending
    lower qubit."""
    pat = "ABCD"[layer % 4]
    edges = []
    for r in range(rows):
        for c in range(cols):
            if pat in "AB" and c + 1 < cols and ((r + c) % 2 == (0 if pat == "A" else 1)):
                edges.append((grid_qubit(r, c, rows), grid_qubit(r, c + 1, rows)))
            if pat in "CD" and r + 1 < rows and ((r + c) % 2 == (0 if pat == "C" else 1)):
                edges.append((grid_qubit(r, c, rows), grid_qubit(r + 1, c, rows)))
    edges.sort(key=lambda e: (min(e), max(e)))
    return edges


def _grid_side(rows: int, cols: int) -> np.ndarray:
    half = cols // 2
    return np.array([0 if (q // rows) < half else 1 for q in range(rows * cols)], dtype=np.uint8)


def _cz_records(edges) -> np.ndarray:
    cz = empty_circuit(len(edges))
    cz["op"] = OP_CZ
    if edges:
        cz["q0"] = [min(e) for e in edges]
        cz["q1"] = [max(e) for e in edges]
    return cz


def grid_circuit(rows: int = 6, cols: int = 8, depth: int = 8, seed: int = 5,
                 max_cross: int | None = 10):
    """Grid circuit with Haar U(2) layers and CZ on four alternating edge
    patterns.  Layer l applies Haar on all qubits then the CZs of pattern
    "ABCD"[l mod 4] (see _grid_pattern_edges).

    The cut separates columns [0, cols/2) from [cols/2, cols).  Only the first
    ``max_cross`` cut-crossing CZs (circuit order) are kept; later crossing
    CZs are dropped.  Returns (gates, side) with side[q] in {0, 1}."""
    rng = _rng(seed)
    n = rows * cols
    side = _grid_side(rows, cols)
    out = []
    kept_cross = 0
    for layer in range(depth):
        g = empty_circuit(n)
        g["op"] = OP_U
        g["q0"] = np.arange(n)
        for q in range(n):
            g["u"][q] = _u_record(haar_u2(rng))
        out.append(g)
        keep = []
        for a, b in _grid_pattern_edges(layer, rows, cols):
            if side[a] != side[b]:
                if max_cross is not None and kept_cross >= max_cross:
                    continue
                kept_cross += 1
            keep.append((a, b))
        out.append(_cz_records(keep))
    return concat(*out), side


def grid_diag_circuit(rows: int = 6, cols: int = 8, depth: int = 8, seed: int = 5,
                      max_cross: int | None = 10):
    """The grid circuit's shape, cut and crossing rule with a closed form at
    every bitstring: one Haar U(2) layer on all qubits, then per layer l a
    T layer (l even) or S layer (l odd) on all qubits followed by the CZs of
    pattern "ABCD"[l mod 4], keeping the first ``max_cross`` crossing CZs.
    Everything after the Haar layer is diagonal, so
    <z|C|0> = prod_q U_q[z_q, 0] * prod of the diagonal gates' phases at z.
    Returns (gates, side)."""
    n = rows * cols
    side = _grid_side(rows, cols)
    out = [haar_layer(n, seed)]
    kept_cross = 0
    for layer in range(depth):
        ph = empty_circuit(n)
        ph["op"] = OP_T if layer % 2 == 0 else OP_S
        ph["q0"] = np.arange(n)
        out.append(ph)
        keep = []
        for a, b in _grid_pattern_edges(layer, rows, cols):
            if side[a] != side[b]:
                if max_cross is not None and kept_cross >= max_cross:
                    continue
                kept_cross += 1
            keep.append((a, b))
        out.append(_cz_records(keep))
    return concat(*out), side


def ghz(n: int) -> np.ndarray:
    """H on qubit 0, then CNOT(i, i+1) for i = 0..n-2 (first argument is the
    control), as in the weak-scaling benchmark circuit of Section 3."""
    g = empty_circuit(n)
    g["op"][0], g["q0"][0] = OP_H, 0
    g["op"][1:] = OP_CNOT
    g["q0"][1:] = np.arange(n - 1)
    g["q1"][1:] = np.arange(1, n)
    return g


def hadamard_all(n: int) -> np.ndarray:
    g = empty_circuit(n)
    g["op"] = OP_H
    g["q0"] = np.arange(n)
    return g


def qft(n: int) -> np.ndarray:
    """Textbook QFT circuit: for j = n-1 down to 0, H on j then CP(2pi/2^(j-k+1))
    controlled by each lower qubit k, followed by swaps that reverse the bit
    order (each swap as three CNOTs).  Maps |x> to
    2^(-n/2) sum_y exp(2 pi i x y / 2^n) |y>."""
    out = []
    for j in range(n - 1, -1, -1):
        out.append(gate(OP_H, j))
        for k in range(j - 1, -1, -1):
            out.append(gate(OP_CP, k, j, theta=2.0 * np.pi / (1 << (j - k + 1))))
    for a in range(n // 2):
        b = n - 1 - a
        out += [gate(OP_CNOT, a, b), gate(OP_CNOT, b, a), gate(OP_CNOT, a, b)]
    return concat(*out)


def prepare_basis(n: int, x: int) -> np.ndarray:
    """X gates that turn |0...0> into |x>."""
    return concat(*[gate(OP_X, q) for q in range(n) if (x >> q) & 1])


def bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    if n >= 63:
        raise ValueError("n < 63 required")
    return rng.integers(0, 1 << n, size=count, dtype=np.uint64)


def cnot_cut_circuit(seed: int):
    """(n, side, gates): 8 qubits cut 4|4, three Haar layers with CNOTs
    across the cut in both directions and one CZ (5 crossing gates)."""
    n = 8
    side = block_parts(n, 2)
    recs = [haar_layer(n, seed)]
    recs += [gate(OP_CNOT, 1, 5), gate(OP_CNOT, 6, 2), gate(OP_CNOT, 0, 1)]
    recs += [haar_layer(n, seed + 1), gate(OP_CZ, 3, 4), gate(OP_CNOT, 7, 0)]
    recs += [haar_layer(n, seed + 2), gate(OP_CNOT, 2, 7), gate(OP_CNOT, 4, 5)]
    return n, side, concat(*recs)


def bitstrings_wide(n: int, count: int, seed: int) -> np.ndarray:
    """count uniform n-bit strings as (count, ceil(n/64)) little-endian uint64
    words (qubit q is bit q % 64 of word q // 64)."""
    words = (n + 63) // 64
    rng = _rng(seed)
    z = rng.integers(0, np.iinfo(np.uint64).max, size=(count, words), dtype=np.uint64,
                     endpoint=True)
    top = n - 64 * (words - 1)
    if top < 64:
        z[:, -1] &= np.uint64((1 << top) - 1)
    return z


def words_to_ints(z: np.ndarray) -> list:
    """Rows of little-endian uint64 words as Python integers."""
    z = np.atleast_2d(np.asarray(z, dtype=np.uint64))
    return [sum(int(w) << (64 * i) for i, w in enumerate(row)) for row in z]


def ints_to_words(zs, n: int) -> np.ndarray:
    """Python integers (< 2^n) as rows of little-endian uint64 words."""
    words = (n + 63) // 64
    out = np.zeros((len(zs), words), dtype=np.uint64)
    for k, z in enumerate(zs):
        for i in range(words):
            out[k, i] = (int(z) >> (64 * i)) & ((1 << 64) - 1)
    return out


def block_parts(n: int, nparts: int) -> np.ndarray:
    """side[q] for nparts blocks of consecutive qubits (sizes differ by at
    most one, lower parts larger)."""
    base, extra = divmod(n, nparts)
    sizes = [base + (1 if p < extra else 0) for p in range(nparts)]
    return np.repeat(np.arange(nparts, dtype=np.uint8), sizes)


def haar_layer(n: int, seed: int) -> np.ndarray:
    """One Haar U(2) gate on every qubit (qubit order)."""
    us = haar_u2_many(_rng(seed), n)
    g = empty_circuit(n)
    g["op"] = OP_U
    g["q0"] = np.arange(n)
    g["u"] = us
    return g


def inverse_circuit_records(gates: np.ndarray) -> np.ndarray:
    """Records of the reversed circuit with every gate replaced by its inverse.
    H, X, Y, Z, CNOT and CZ are self-inverse; S, T and U become OP_U with the
    conjugate transpose; CP(theta) becomes CP(-theta).  (Record manipulation
    for round-trip tests: conjugate-transposing a literal 2x2 is not a
    simulation step.)"""
    inv = gates[::-1].copy()
    for k in range(len(inv)):
        op = int(inv["op"][k])
        if op == OP_S:
            inv[k] = gate(OP_U, int(inv["q0"][k]), u=np.diag([1.0, -1j]))[0]
        elif op == OP_T:
            inv[k] = gate(OP_U, int(inv["q0"][k]), u=np.diag([1.0, np.exp(-0.25j * np.pi)]))[0]
        elif op == OP_U:
            m = inv["u"][k].reshape(2, 2, 2)
            m = m[..., 0] + 1j * m[..., 1]
            inv["u"][k] = _u_record(m.conj().T)
        elif op == OP_CP:
            inv["theta"][k] = -inv["theta"][k]
    return inv


# Named workload sizes ------------------------------------------------------
def workload_mixed20():
    """n=20, 200 mixed gates (seed 1); full state + norm."""
    return 20, random_mixed(20, 200, seed=1)


def workload_brick30():
    """n=30, 20 brick layers (seed 2), 4096 bitstrings (seed 1002)."""
    return 30, layered_brick(30, 20, seed=2), bitstrings(30, 4096, seed=1002)


def workload_brick(n: int, layers: int, seed: int = 3):
    return n, layered_brick(n, layers, seed=seed)
