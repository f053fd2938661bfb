"""GPU parity of the batched graph launch and of the Eq. (3) branch
driver against the oracle."""
import math
import os
import sys

import numpy as np
import pytest

from _parity import assert_c64, rel_l2
from oracle import decomposition as odec
from oracle import statevector as sv
from paper_1912_03243_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import GRID_SETS, load, path_for  # noqa: E402

pytestmark = pytest.mark.gpu



def parts_circuit(nparts, seed):
    """nparts parts of three qubits: Haar U(2) layers, a CZ inside every part
    and 5 CZs between parts (32 branches)."""
    rng = np.random.default_rng(seed)
    n = 3 * nparts
    side = np.arange(n) // 3
    recs = []
    cross = [(0, 3), (1, 4 if nparts > 2 else 5), (2, 6), (4, 7), (3, 3 * nparts - 1)]
    for layer in range(3):
        recs += [W.gate(W.OP_U, q, u=W.haar_u2(rng)) for q in range(n)]
        recs += [W.gate(W.OP_CZ, 3 * p, 3 * p + 1 + layer % 2) for p in range(nparts)]
        if layer < 2:
            recs += [W.gate(W.OP_CZ, a, b) for a, b in cross[layer * 2: layer * 2 + 2 + layer]]
    return n, side, W.concat(*recs)

@pytest.fixture(scope="module")
def J():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03243_amd import juqcs
    return juqcs


def announce(*what):
    print("CASE", *what, flush=True)


def mixed_batch(seed=0):
    rng = np.random.default_rng(seed)
    circuits = []
    for i, n in enumerate([1, 3, 5, 8, 12, 13, 14, 15, 17, 13, 16]):
        if i % 2:
            circ = W.layered_random_pairs(n, int(rng.integers(2, 6)), rng)
        else:
            circ = W.random_mixed(n, 60, seed=100 + i, p1=1.0 if n == 1 else 0.6)
        circuits.append((n, circ))
    circuits.append((9, W.empty_circuit(0)))            # no gates: |0...0>
    return circuits


@pytest.mark.parametrize("fuse_k", [0, 1, 2, 3, 4])
def test_batch_matches_oracle(J, fuse_k):
    announce("batch", fuse_k)
    circuits = mixed_batch()
    b = J.Batch(circuits, fuse_k=fuse_k)
    b.run()
    b.wait()
    st = b.stats()
    assert st["gate_apps"] == sum(len(c) for _, c in circuits)
    for i, (n, circ) in enumerate(circuits):
        assert_c64(b.state_vector(i), sv.run_circuit(n, circ))
    if fuse_k:
        assert np.all(b.fusion() == fuse_k)
    b.close()


@pytest.mark.parametrize("relabel", [-1, 0])
def test_batch_relabel(J, relabel):
    # deep circuits on 16-20 qubits need several passes; with relabeling the
    # passes move qubits onto the low bits and the readouts map through the
    # recorded layout
    announce("batch-relabel", relabel)
    circuits = [(n, W.layered_brick(n, 10, seed=300 + n)) for n in (16, 17, 18, 20)]
    circuits.append((19, W.random_mixed(19, 150, seed=319)))
    b = J.Batch(circuits, relabel=relabel)
    b.run()
    b.wait()
    z = np.stack([np.arange(0, 1 << 16, 331, dtype=np.uint64)[:150]] * len(circuits))
    amps = b.amplitudes(z)
    moved = 0
    for i, (n, circ) in enumerate(circuits):
        phi = sv.run_circuit(n, circ)
        assert_c64(b.state_vector(i), phi)
        assert_c64(amps[i], phi[z[i].astype(np.int64)])
        layout = b.layout(i)
        assert sorted(layout) == list(range(n))
        moved += layout != list(range(n))
    assert moved > 0 if relabel == 0 else moved == 0
    b.close()


def test_batch_graph_replay_and_readout(J):
    import torch
    announce("batch-graph")
    circuits = mixed_batch(1)
    s = torch.cuda.Stream()
    b = J.Batch(circuits)
    with torch.cuda.stream(s):
        b.run(s)
        b.wait()
        first = [b.state_vector(i) for i in range(len(circuits))]
        b.states.fill_(7)                       # garbage: every run starts from |0...0>
        for _ in range(3):                      # graph replays
            b.run(s)
            b.wait()
            torch.cuda.synchronize()
            for i in range(len(circuits)):
                assert np.array_equal(b.state_vector(i), first[i])
        idx = np.stack([np.arange(8, dtype=np.uint64) % (1 << n) for n, _ in circuits])
        amps = b.amplitudes(idx, s)
        norms = b.norms(s)
    for i, (n, circ) in enumerate(circuits):
        phi = sv.run_circuit(n, circ)
        assert np.allclose(amps[i], phi[idx[i].astype(np.int64)], atol=1e-6)
        assert abs(norms[i] - 1.0) < 1e-5
    b.close()


def test_batch_order_does_not_change_results(J):
    announce("batch-order")
    circuits = mixed_batch(2)
    perm = np.random.default_rng(3).permutation(len(circuits))
    b1 = J.Batch(circuits, fuse_k=2)
    b2 = J.Batch([circuits[i] for i in perm], fuse_k=2)
    b1.run()
    b2.run()
    b1.wait()
    b2.wait()
    for j, i in enumerate(perm):
        assert np.array_equal(b1.state_vector(int(i)), b2.state_vector(j))


def test_batch_autotune(J):
    announce("batch-autotune")
    rng = np.random.default_rng(9)
    circuits = [(n, W.layered_random_pairs(n, 6, rng)) for n in (12, 14, 16, 12, 14)]
    b = J.Batch(circuits, autotune=True)
    k = b.fusion()
    assert np.all((k >= 1) & (k <= 4))
    assert k[0] == k[3] and k[1] == k[4]      # one choice per qubit count
    b.run()
    b.wait()
    for i, (n, circ) in enumerate(circuits):
        assert_c64(b.state_vector(i), sv.run_circuit(n, circ))


def test_batch_rejects_bad_input(J):
    with pytest.raises(J.JuqcsError) as e:
        J.Batch([(3, W.concat(W.gate(W.OP_CZ, 0, 3)))])
    assert e.value.status == J.ERR_QUBIT
    with pytest.raises(J.JuqcsError):
        J.Batch([(31, W.empty_circuit(0))], states=__import__("torch").empty(16, device="cuda"))


# ---- Eq. (3): branch sums -------------------------------------------------------------
@pytest.mark.parametrize("rows, cols, depth, seed, group", [(2, 4, 4, 3, 0), (4, 4, 8, 9, 3),
                                                           (2, 6, 6, 1, 0), (4, 6, 6, 2, 5)])
def test_branch_amplitudes_small_grids(J, rows, cols, depth, seed, group):
    announce("branch", rows, cols, depth, seed, group)
    circ, side = W.grid_circuit(rows, cols, depth, seed, max_cross=None)
    n = rows * cols
    z = np.random.default_rng(seed).integers(0, 1 << n, 40, dtype=np.uint64)
    got = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=group)
    ob = odec.branch_amplitudes(n, circ, side, z[:8])
    scale = np.abs(ob).max()
    assert np.max(np.abs(got[:8] - ob)) / scale < 1e-5
    if n <= 16:  # and to the full state vector
        full = sv.run_circuit(n, circ)
        want = full[z.astype(np.int64)]
        assert np.max(np.abs(got - want)) / np.abs(full).max() < 1e-5


@pytest.mark.parametrize("nparts, seed, group", [(3, 5, 0), (4, 6, 3), (3, 7, 1)])
def test_branch_amplitudes_more_parts(J, nparts, seed, group):
    # P > 2 parts (Section 4's general partition): against the oracle's
    # branch sum and the full state vector
    announce("branch-parts", nparts, seed, group)
    n, side, circ = parts_circuit(nparts, seed)
    side = side.astype(np.uint8)
    z = np.random.default_rng(seed).integers(0, 1 << n, 40, dtype=np.uint64)
    got = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=group)
    ob = odec.branch_amplitudes(n, circ, side, z[:8])
    full = sv.run_circuit(n, circ)
    scale = np.abs(full).max()
    assert np.max(np.abs(got[:8] - ob)) / scale < 1e-5
    assert np.max(np.abs(got - full[z.astype(np.int64)])) / scale < 1e-5


@pytest.mark.parametrize("group", [0, 2])
def test_branch_every_coefficient(J, group):
    # all 2^16 coefficients of a 16-qubit grid at once (the gathered
    # amplitudes of a branch group scale with their count), against the
    # full state vector; the sum runs in branch order, so the group size
    # changes nothing
    announce("branch-all", group)
    circ, side = W.grid_circuit(4, 4, 8, 11, max_cross=4)
    n = 16
    z = np.arange(1 << n, dtype=np.uint64)
    got = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=group)
    full = sv.run_circuit(n, circ)
    assert np.max(np.abs(got - full)) / np.abs(full).max() < 1e-5
    if group:
        ref = J.juqcs_branch_amplitudes(n, circ, side, z)
        assert np.array_equal(got, ref)


def test_branch_sum_paths_agree(J):
    # a group of more than 48 distinct part states is summed from where the
    # states lie, a smaller one from LDS: same arithmetic in the same order,
    # so the same bits
    announce("branch-sum-paths")
    circ, side = W.grid_circuit(4, 4, 6, 3, max_cross=None)
    n = 16
    assert len(odec.crossing_gates(circ, side)) >= 5   # 2 parts x 2^m states > 48
    z = np.random.default_rng(3).integers(0, 1 << n, 300, dtype=np.uint64)
    big = J.juqcs_branch_amplitudes(n, circ, side, z)
    small = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=4)
    assert np.array_equal(big, small)
    full = sv.run_circuit(n, circ)
    assert_c64(big, full[z.astype(np.int64)])


def test_branch_rejects_too_many_parts(J):
    side = np.arange(9, dtype=np.uint8)  # 9 parts
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_branch_amplitudes(9, W.concat(W.gate(W.OP_H, 0)), side, [0])
    assert e.value.status == J.ERR_ARG


def test_branch_ghz48_closed_form(J, golden):
    n = 48
    announce("branch-ghz48")
    recs = [W.gate(W.OP_H, 0)]
    for i in range(n - 1):
        if i == n // 2 - 1:                      # the crossing CNOT as H_t CZ H_t
            recs += [W.gate(W.OP_H, i + 1), W.gate(W.OP_CZ, i, i + 1), W.gate(W.OP_H, i + 1)]
        else:
            recs.append(W.gate(W.OP_CNOT, i, i + 1))
    side = np.array([0] * 24 + [1] * 24, dtype=np.uint8)
    z = np.array([0, (1 << n) - 1, 1, 1 << 47, 12345], dtype=np.uint64)
    got = J.juqcs_branch_amplitudes(n, W.concat(*recs), side, z)
    assert abs(got[0] - golden["ghz.amp_all_zero"]) < 1e-6
    assert abs(got[1] - golden["ghz.amp_all_one"]) < 1e-6
    assert np.all(np.abs(got[2:]) < 1e-7)


@pytest.mark.parametrize("name", ["grid48m2", "grid42m3"])
@pytest.mark.parametrize("group", [0, 1, 2])
def test_branch_grid_against_stored_oracle_values(J, name, group):
    # full-size halves (24 and 21 qubits) against the oracle's own branch
    # sum, with every branch in one group and in groups of one and two
    if not os.path.exists(path_for(name)):
        pytest.skip("stored amplitudes not generated")
    rows, cols, depth, seed, mcross, _, _ = GRID_SETS[name]
    z, want = load(name)
    circ, side = W.grid_circuit(rows, cols, depth, seed, max_cross=mcross)
    announce(name, group)
    got = J.juqcs_branch_amplitudes(rows * cols, circ, side, z, group_size=group)
    assert rel_l2(got, want) < 1e-5
    assert np.max(np.abs(got - want)) / np.abs(want).max() < 1e-5


def test_branch_rejects_other_crossings(J):
    # only CZ and CNOT are decomposed: a controlled phase across the cut is not
    side = np.array([0, 0, 1, 1], dtype=np.uint8)
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_branch_amplitudes(4, W.concat(W.gate(W.OP_CP, 1, 2, theta=0.3)), side, [0])
    assert e.value.status == J.ERR_UNSUPPORTED


@pytest.mark.parametrize("seed, group", [(11, 0), (12, 2)])
def test_branch_crossing_cnots(J, seed, group):
    # CNOTs across the cut in both directions (each its CZ between Hadamards
    # on the target) and a CZ: all 256 coefficients against the full state
    # vector and the oracle's branch sum
    announce("branch-cnot", seed, group)
    n, side, circ = W.cnot_cut_circuit(seed)
    z = np.arange(1 << n, dtype=np.uint64)
    got = J.juqcs_branch_amplitudes(n, circ, side, z, group_size=group)
    full = sv.run_circuit(n, circ)
    assert_c64(got, full)
    ob = odec.branch_amplitudes(n, circ, side, z[:16])
    assert np.max(np.abs(got[:16] - ob)) / np.abs(full).max() < 1e-5


def test_branch_ghz128_paper_values(J, golden):
    # Section 4's scaling circuit at its largest size: GHZ on 128 qubits in
    # eight parts of 16 (7 crossing CNOTs, 128 branches).  |0...0> and
    # |1...1> have 1/sqrt(2); strings with uniform parts that differ cancel
    # in the branch sum; every other string is exactly zero.
    n = 128
    announce("branch-ghz128")
    side = W.block_parts(n, 8)
    ones = (1 << n) - 1
    mixed = [sum(((1 << 16) - 1) << (16 * p) for p in range(8) if (m >> p) & 1)
             for m in (0b00000001, 0b10110010, 0b01111111, 0b10000000)]
    head = W.ints_to_words([0, ones] + mixed, n)
    z = np.concatenate([head, W.bitstrings_wide(n, 1 << 16, 5)])
    got = J.juqcs_branch_amplitudes(n, W.ghz(n), side, z)
    assert abs(got[0] - golden["ghz.amp_all_zero"]) < 1e-6
    assert abs(got[1] - golden["ghz.amp_all_one"]) < 1e-6
    assert np.max(np.abs(got[2:6])) < 1e-6
    assert np.all(got[6:] == 0)


def ghz_blocks(n, blocks):
    """H on the first qubit of every block [a, b) of consecutive qubits, then
    the CNOT chain a -> a+1 -> ... -> b-1: a product of GHZ states."""
    recs = []
    for a, b in blocks:
        recs.append(W.gate(W.OP_H, a))
        recs += [W.gate(W.OP_CNOT, i, i + 1) for i in range(a, b - 1)]
    return W.concat(*recs)


def ghz_haar_closed_form(layer, zs, n, blocks):
    """prod over blocks of (prod_q U_q[z_q, 0] + prod_q U_q[z_q, 1]) / sqrt(2):
    the coefficient at z of U_0 (x) ... (x) U_{n-1} applied to the product of
    the blocks' GHZ states."""
    u = layer["u"].reshape(n, 2, 2, 2)
    u = u[..., 0] + 1j * u[..., 1]
    out = []
    for z in zs:
        amp = 1.0 + 0.0j
        for a, b in blocks:
            a0 = np.prod([u[q, (z >> q) & 1, 0] for q in range(a, b)])
            a1 = np.prod([u[q, (z >> q) & 1, 1] for q in range(a, b)])
            amp *= (a0 + a1) / math.sqrt(2.0)
        out.append(amp)
    return np.array(out)


# n = 100 puts a part across the 64-bit word boundary; n = 240 is eight parts
# of 30 qubits (8 GiB part states) with two crossing CNOTs
WIDE_CASES = [(96, 6, 0, [(0, 96)]), (100, 5, 3, [(0, 100)]), (128, 8, 0, [(0, 128)]),
              (240, 8, 0, [(0, 30), (30, 65), (65, 90), (90, 120), (120, 150), (150, 185),
                           (185, 210), (210, 240)])]


@pytest.mark.parametrize("n, nparts, group, blocks", WIDE_CASES)
def test_branch_wide_ghz_haar_closed_form(J, n, nparts, group, blocks):
    # GHZ states followed by a Haar U(2) on every qubit have a closed form
    # at any z
    announce("branch-wide", n, nparts, group)
    layer = W.haar_layer(n, 21)
    circ = W.concat(ghz_blocks(n, blocks), layer)
    side = W.block_parts(n, nparts)
    zs = W.words_to_ints(W.bitstrings_wide(n, 62, 22)) + [0, (1 << n) - 1]
    got = J.juqcs_branch_amplitudes(n, circ, side, W.ints_to_words(zs, n), group_size=group)
    assert_c64(got, ghz_haar_closed_form(layer, zs, n, blocks))
    if n == 96:  # and the oracle's branch sum
        ob = odec.branch_amplitudes(n, circ, side, zs[:3])
        assert_c64(got[:3], ob)


def test_branch_wide_matches_narrow(J):
    # the same bitstrings as one word each: identical results
    announce("branch-wide-narrow")
    n, side, circ = parts_circuit(3, 5)
    side = side.astype(np.uint8)
    z = np.random.default_rng(5).integers(0, 1 << n, 64, dtype=np.uint64)
    a = J.juqcs_branch_amplitudes(n, circ, side, z)
    b = J.juqcs_branch_amplitudes(n, circ, side, z.reshape(-1, 1))
    c = J.juqcs_branch_amplitudes(n, circ, side, np.stack([z, np.zeros_like(z)], axis=1))
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_branch_without_crossings_and_empty(J):
    # no gate crosses the parts (one branch, m = 0): a product state, whose
    # coefficient is prod_q U_q[z_q, 0]; and no bitstrings at all
    announce("branch-m0")
    n = 30
    layer = W.haar_layer(n, 31)
    side = W.block_parts(n, 3)
    zs = W.words_to_ints(W.bitstrings_wide(n, 32, 32)) + [0, (1 << n) - 1]
    got = J.juqcs_branch_amplitudes(n, layer, side, np.array(zs, dtype=np.uint64))
    u = layer["u"].reshape(n, 2, 2, 2)
    u = u[..., 0] + 1j * u[..., 1]
    want = np.array([np.prod([u[q, (z >> q) & 1, 0] for q in range(n)]) for z in zs])
    assert_c64(got, want)
    assert J.juqcs_branch_amplitudes(n, layer, side, np.zeros(0, dtype=np.uint64)).size == 0


def test_branch_device_matches_host(J):
    # bitstrings and result in device memory: the same kernels, the same bits
    import torch
    announce("branch-device")
    n, nparts = 100, 5
    circ = W.concat(ghz_blocks(n, [(0, n)]), W.haar_layer(n, 21))
    side = W.block_parts(n, nparts)
    z = W.bitstrings_wide(n, 4096, 23)
    host = J.juqcs_branch_amplitudes(n, circ, side, z)
    dz = torch.from_numpy(z.view(np.int64)).cuda()
    out = torch.empty(2 * z.shape[0], dtype=torch.float64, device="cuda")
    J.juqcs_branch_amplitudes_device(n, circ, side, dz, out)
    dev = out.cpu().numpy().view(np.complex128)
    assert np.array_equal(dev, host)


def test_branch_device_rejects_bits_above_n(J):
    import torch
    n = 100
    z = np.zeros((8, 2), dtype=np.uint64)
    z[5, 1] = np.uint64(1 << 40)  # qubit 104
    dz = torch.from_numpy(z.view(np.int64)).cuda()
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_branch_amplitudes_device(n, W.ghz(n), W.block_parts(n, 5), dz, out)
    assert e.value.status == J.ERR_ARG


@pytest.mark.parametrize("n, words, top", [(100, 2, 1 << 40), (128, 1, 0), (241, 4, 0)])
def test_branch_wide_rejects(J, n, words, top):
    # a bit at or above n, too few words, more than 240 qubits
    side = W.block_parts(n, 8) if n <= 240 else np.zeros(n, dtype=np.uint8)
    z = np.zeros((1, words), dtype=np.uint64)
    z[0, -1] = top
    with pytest.raises(J.JuqcsError) as e:
        J.juqcs_branch_amplitudes(n, W.ghz(n), side, z)
    assert e.value.status == J.ERR_ARG
