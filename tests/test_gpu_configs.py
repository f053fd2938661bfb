"""GPU parity of the configurations at their stated sizes: the 20-qubit mixed
circuit (full state), a parsed OpenQASM program, the 48-qubit grid
decomposition at m = 10 against a closed form, the branch sums' two
summation paths, and a stratified oracle sample of the 4096-circuit batch.

Every case prints its name before the GPU work so a failing run names it.
"""
import cmath
import math
import os
import sys

import numpy as np
import pytest

from _closed_forms import diag_closed_form
from _parity import assert_c128, assert_c64, rel_l2
from oracle import decomposition as odec
from oracle import statevector as sv
from paper_1912_03243_amd import qasm
from paper_1912_03243_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import load_batch, path_for  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03243_amd import juqcs
    return juqcs


def announce(*what):
    print("CASE", *what, flush=True)


# ---- the 20-qubit mixed circuit: full state and norm ----------------------------------
@pytest.fixture(scope="module")
def mixed20():
    n, circ = W.workload_mixed20()
    return n, circ, sv.run_circuit(n, circ)


@pytest.mark.parametrize("mode", ["plain", "tile"])
def test_mixed20_full_state(J, mixed20, mode):
    n, circ, phi = mixed20
    announce("mixed20", mode)
    with J.State(n, "c128") as s:
        s.init(0)
        o = s.run(circ, mode=mode)
        nrm = s.norm()
        s.canonicalize()
        got = s.state_vector()
    assert o.gates == 200
    assert_c128(got, phi)
    assert abs(nrm - sv.norm(phi)) <= 1e-12


def test_mixed20_c64_full_state(J, mixed20):
    n, circ, phi = mixed20
    announce("mixed20 c64 tile")
    with J.State(n, "c64") as s:
        s.init(0)
        s.run(circ, mode="tile")
        got = s.state_vector()
    assert_c64(got, phi)


# ---- an OpenQASM program through the library ---------------------------------------------
def qft_program(n, x):
    """Basis state |x> (x gates) followed by the textbook QFT: H and
    controlled phases cu1(pi / 2^(j-k)) from the top qubit down, then the
    swaps that reverse the bit order."""
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n}];", f"creg c[{n}];"]
    lines += [f"x q[{q}];" for q in range(n) if (x >> q) & 1]
    for j in range(n - 1, -1, -1):
        lines.append(f"h q[{j}];")
        for k in range(j - 1, -1, -1):
            lines.append(f"cu1(pi/{1 << (j - k)}) q[{k}],q[{j}];")
    lines += [f"swap q[{a}],q[{n - 1 - a}];" for a in range(n // 2)]
    lines.append("barrier q;")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("n, x, mode", [(12, 0x5a3, "plain"), (12, 0x5a3, "tile"), (18, 77777, "tile")])
def test_qasm_qft_of_basis_state(J, n, x, mode):
    # QFT|x> = 2^(-n/2) sum_y exp(2 pi i x y / 2^n) |y>  (closed form at any n)
    announce("qasm-qft", n, x, mode)
    m, gates = qasm.parse_qasm(qft_program(n, x))
    assert m == n
    with J.State(n, "c128") as s:
        s.init(0)
        s.run(gates, mode=mode)
        got = s.state_vector()
    y = np.arange(1 << n, dtype=np.float64)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    assert_c128(got, want)
    if n <= 12:
        assert_c128(got, sv.run_circuit(n, gates))


# ---- Eq. (3) at the 48-qubit grid's own shape, cut and m = 10 -----------------------------
def test_grid48_m10_closed_form_all_sum_paths(J):
    # 1024 branch pairs of 24-qubit halves; 2^16 + 4 coefficients, so the sum
    # from global memory runs in chunks.  group 16: 32 leaves, summed from
    # LDS; group 64: 128 leaves, summed from global memory; group 0: as many
    # as fit.  Same arithmetic in the same order: identical bits.
    n, m = 48, 10
    circ, side = W.grid_diag_circuit(6, 8, 8, seed=5, max_cross=m)
    assert len(odec.crossing_gates(circ, side)) == m
    z = np.concatenate([np.array([0, (1 << n) - 1, 1, 1 << 47], dtype=np.uint64),
                        W.bitstrings(n, 1 << 16, seed=1005)])
    want = diag_closed_form(circ, n, z)
    got = {}
    for group in (16, 64, 0):
        announce("grid48-m10", group)
        got[group] = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=group)
        err = float(np.max(np.abs(got[group] - want)) / np.abs(want).max())
        print(f"grid48 m=10 group={group}: max|err|/max|a| = {err:.3e}, "
              f"rel L2 = {rel_l2(got[group], want):.3e}", flush=True)
    for group in (16, 64, 0):
        assert_c64(got[group], want)
    assert np.array_equal(got[16], got[64]) and np.array_equal(got[16], got[0])


@pytest.mark.parametrize("m", [2, 4, 6, 8])
def test_grid48_closed_form_fewer_crossings(J, m):
    # the error of the branch sum against the number of decomposed CZs
    n = 48
    circ, side = W.grid_diag_circuit(6, 8, 8, seed=5, max_cross=m)
    z = W.bitstrings(n, 4096, seed=1005)
    announce("grid48-closed", m)
    got = J.juqcs_branch_amplitudes(n, circ, side, z)
    want = diag_closed_form(circ, n, z)
    print(f"grid48 m={m}: max|err|/max|a| = "
          f"{float(np.max(np.abs(got - want)) / np.abs(want).max()):.3e}, "
          f"rel L2 = {rel_l2(got, want):.3e}", flush=True)
    assert_c64(got, want)


def three_part_circuit(seed):
    """Three parts of four qubits with Haar layers and 9 crossing CZs between
    every pair of parts (each part on 6 of them: 2^6 leaves per part when all
    branches form one group, more than the LDS sum holds)."""
    rng = np.random.default_rng(seed)
    n = 12
    side = (np.arange(n) // 4).astype(np.uint8)
    cross = [(0, 4), (1, 8), (5, 9), (2, 6), (3, 10), (7, 11), (0, 9), (4, 8), (1, 6)]
    recs = []
    for layer in range(3):
        recs.append(W.haar_layer(n, int(rng.integers(1 << 30))))
        recs += [W.gate(W.OP_CZ, 4 * p, 4 * p + 1 + layer % 3) for p in range(3)]
        recs += [W.gate(W.OP_CZ, a, b) for a, b in cross[3 * layer: 3 * layer + 3]]
    recs.append(W.haar_layer(n, int(rng.integers(1 << 30))))
    return n, side, W.concat(*recs)


def test_branch_three_parts_sum_paths_bit_identical(J):
    # P = 3: the global-memory sum (one group of 512 branches: 3 x 64 leaves),
    # in chunks (2^16 coefficients), and the LDS sum (groups of 4 branches)
    # give the same bits, and both match the full state vector
    n, side, circ = three_part_circuit(17)
    assert len(odec.crossing_gates(circ, side)) == 9
    z = np.random.default_rng(18).integers(0, 1 << n, 1 << 16, dtype=np.uint64)
    announce("branch-3parts-paths")
    glob = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=512)
    lds = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=4)
    assert np.array_equal(glob, lds)
    full = sv.run_circuit(n, circ)
    assert_c64(glob, full[z.astype(np.int64)])


# ---- the 4096-circuit batch against stored oracle amplitudes -------------------------------
def test_batch4096_stratified_oracle_sample(J):
    # the batch configuration as a whole (4096 circuits, one graph launch);
    # a stratified sample with every qubit count 12..24 (22 circuits, 64
    # seeded amplitudes each) against the oracle's full state vectors
    if not os.path.exists(path_for("batch4096s")):
        pytest.skip("stored batch amplitudes not generated")
    import torch
    ref = load_batch("batch4096s")
    inst = W.batch_instances(4096)
    announce("batch4096", len(ref))
    b = J.Batch(inst)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(s)
        b.wait()
        idx = np.stack([W.batch_bitstrings(i, n) for i, (n, _) in enumerate(inst)])
        amps = b.amplitudes(idx, s)
        norms = b.norms(s)
    b.close()
    del b
    torch.cuda.empty_cache()
    assert np.max(np.abs(norms - 1.0)) < 1e-5
    worst = 0.0
    for i, (z, want) in ref.items():
        assert np.array_equal(idx[i], z)
        worst = max(worst, rel_l2(amps[i], want))
        assert_c64(amps[i], want)
    print(f"batch4096 sample: {len(ref)} circuits, worst rel L2 {worst:.3e}", flush=True)
