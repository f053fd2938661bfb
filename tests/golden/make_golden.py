"""Writes the stored expected amplitudes used by the full-size GPU tests.

Calls only the CPU oracle (and the seeded workload generators).  The
amplitudes of a 28-36 qubit layered circuit are far too many for the oracle's
full state-vector path, so each requested coefficient is computed with the
paper's entangling-gate decomposition (Section 4, Eq. (3)): the qubits are cut
into a low and a high half, every CZ across the cut is split with Eq. (2),
and <z|C|0> = 2^-S sum_s A_s(z_low) B_s(z_high) in FP64.  The decomposition
is pinned against the full state vector in tests/test_oracle_pins.py.

The batch sample (batch4096s) takes a stratified sample of the 4096 batched
circuits -- every qubit count 12..24, the shallowest circuit for n >= 21 and
the first and the deepest for n <= 20 -- and stores 64 seeded amplitudes of
each, from the oracle's full state vector.

usage: python tests/golden/make_golden.py brick30 [brick28 brick34 brick36 grid48m2 grid42m3
                                                   batch4096s]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import decomposition  # noqa: E402
from paper_1912_03243_amd import workloads as W  # noqa: E402

# name: (n, layers, circuit seed, bitstring seed, count)
# grid48m2: the 6x8 grid circuit (depth 8, seed 5) keeping only its first two
# cut-crossing CZs, amplitudes by Eq. (3) over the 24|24 column cut.
# grid42m3: the 7x6 grid circuit (depth 12, seed 7) keeping its first three,
# over the 21|21 column cut.
GRID_SETS = {"grid48m2": (6, 8, 8, 5, 2, 1005, 64), "grid42m3": (7, 6, 12, 7, 3, 1007, 64)}
SETS = {
    "brick30": (30, 20, 2, 1002, 256),
    "brick28": (28, 16, 3, 1003, 256),
    "brick34": (34, 16, 3, 1003, 256),
    "brick36": (36, 16, 3, 1003, 256),
}


BATCH_COUNT = 4096
BATCH_AMPS = 64


def batch_sample(count=BATCH_COUNT):
    """Indices of the stored batch circuits: for every qubit count, the
    shallowest instance when n >= 21 (the oracle's full state costs most
    there), else the first and the deepest one."""
    shapes = [W.batch_shape(i) for i in range(count)]
    pick = []
    for n in sorted({s[0] for s in shapes}):
        idx = [i for i, s in enumerate(shapes) if s[0] == n]
        deepest = max(idx, key=lambda i: (shapes[i][1], -i))
        shallowest = min(idx, key=lambda i: (shapes[i][1], i))
        pick += [shallowest] if n >= 21 else sorted({idx[0], deepest})
    return sorted(pick)


def make_batch(name):
    from oracle import statevector as sv
    sample = batch_sample()
    t0 = time.time()
    with open(path_for(name), "w") as f:
        f.write(f"# {name}: batch_instance(i) of the {BATCH_COUNT}-circuit batch for a stratified "
                f"sample of i; batch_bitstrings(i, n, {BATCH_AMPS})\n")
        f.write("# amplitudes from the FP64 oracle's full state vector (statevector.run_circuit)\n")
        f.write("# i z re im\n")
        for i in sample:
            n, circ = W.batch_instance(i)
            z = W.batch_bitstrings(i, n, BATCH_AMPS)
            t1 = time.time()
            psi = sv.run_circuit(n, circ)
            for zi in z:
                a = psi[int(zi)]
                f.write(f"{i} {int(zi)} {a.real:.17e} {a.imag:.17e}\n")
            f.flush()
            print(f"  circuit {i}: n={n} gates={len(circ)} {time.time() - t1:.1f}s", flush=True)
    print(f"{name}: {len(sample)} circuits {time.time() - t0:.1f}s -> {path_for(name)}", flush=True)


def load_batch(name="batch4096s"):
    """{circuit index: (z uint64 array, complex128 amplitudes)}."""
    out = {}
    with open(path_for(name)) as f:
        for line in f:
            if line.startswith("#"):
                continue
            i, z, re, im = line.split()
            zs, am = out.setdefault(int(i), ([], []))
            zs.append(int(z))
            am.append(float(re) + 1j * float(im))
    return {i: (np.array(z, dtype=np.uint64), np.array(a)) for i, (z, a) in out.items()}


def path_for(name):
    return os.path.join(HERE, f"{name}_amplitudes.txt")


def make_grid(name):
    rows, cols, depth, cseed, mcross, zseed, count = GRID_SETS[name]
    circ, side = W.grid_circuit(rows, cols, depth, cseed, max_cross=mcross)
    n = rows * cols
    z = W.bitstrings(n, count, seed=zseed)
    S = len(decomposition.crossing_gates(circ, side))
    t0 = time.time()
    amps = decomposition.branch_amplitudes(n, circ, side, z)
    dt = time.time() - t0
    with open(path_for(name), "w") as f:
        f.write(f"# {name}: grid_circuit(rows={rows}, cols={cols}, depth={depth}, seed={cseed}, "
                f"max_cross={mcross}); bitstrings(n={n}, count={count}, seed={zseed})\n")
        f.write(f"# <z|C|0> by Eq. (3) (Section 4) over the column cut, S={S}, FP64 oracle, "
                f"{dt:.0f} s\n")
        f.write("# z re im\n")
        for zi, a in zip(z, amps):
            f.write(f"{int(zi)} {a.real:.17e} {a.imag:.17e}\n")
    print(f"{name}: S={S} {dt:.1f}s -> {path_for(name)}", flush=True)


def make(name):
    if name == "batch4096s":
        return make_batch(name)
    if name in GRID_SETS:
        return make_grid(name)
    n, layers, cseed, zseed, count = SETS[name]
    circ = W.layered_brick(n, layers, seed=cseed)
    z = W.bitstrings(n, count, seed=zseed)
    side = np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.uint8)
    S = len(decomposition.crossing_gates(circ, side))
    t0 = time.time()
    amps = decomposition.branch_amplitudes(n, circ, side, z)
    dt = time.time() - t0
    with open(path_for(name), "w") as f:
        f.write(f"# {name}: layered_brick(n={n}, layers={layers}, seed={cseed}); "
                f"bitstrings(n={n}, count={count}, seed={zseed})\n")
        f.write(f"# <z|C|0> by Eq. (3) (Section 4) with the cut {n // 2}|{n - n // 2}, "
                f"S={S} decomposed CZs, FP64 oracle, {dt:.0f} s\n")
        f.write("# z re im\n")
        for zi, a in zip(z, amps):
            f.write(f"{int(zi)} {a.real:.17e} {a.imag:.17e}\n")
    print(f"{name}: S={S} {dt:.1f}s -> {path_for(name)}", flush=True)


def load(name):
    z, re, im = [], [], []
    with open(path_for(name)) as f:
        for line in f:
            if line.startswith("#"):
                continue
            a, b, c = line.split()
            z.append(int(a))
            re.append(float(b))
            im.append(float(c))
    return np.array(z, dtype=np.uint64), np.array(re) + 1j * np.array(im)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["brick30"]:
        make(nm)
