"""Host-side checks of the seeded workload generators (no GPU)."""
import numpy as np

from oracle import decomposition as dec
from paper_1912_03243_amd import workloads as W


def test_brick_gate_counts():
    for n, layers, total in [(30, 20, 890), (34, 16, 808), (36, 16, 856), (28, 16, 664)]:
        g = W.layered_brick(n, layers, seed=3)
        assert len(g) == total
        assert np.sum(g["op"] == W.OP_CZ) == total - n * layers


def test_generators_are_deterministic():
    a = W.layered_brick(12, 4, seed=2)
    b = W.layered_brick(12, 4, seed=2)
    assert a.tobytes() == b.tobytes()
    assert W.bitstrings(30, 16, 1002).tolist() == W.bitstrings(30, 16, 1002).tolist()


def test_haar_matrices_are_unitary():
    g = W.layered_brick(8, 2, seed=9)
    for rec in g[g["op"] == W.OP_U]:
        m = rec["u"].reshape(2, 2, 2)
        m = m[..., 0] + 1j * m[..., 1]
        assert np.allclose(m.conj().T @ m, np.eye(2), atol=1e-14)


def test_grid_cut_has_ten_crossing_czs():
    g, side = W.grid_circuit()
    assert len(dec.crossing_gates(g, side)) == 10
    assert side.tolist() == [0] * 24 + [1] * 24
    full, _ = W.grid_circuit(max_cross=None)
    assert len(dec.crossing_gates(full, side)) == 12
    assert len(full) - len(g) == 2


def test_batch_instance_ranges():
    inst = W.batch_instances(64)
    ns = [n for n, _ in inst]
    assert min(ns) >= 12 and max(ns) <= 24
    for n, g in inst:
        assert np.all(g["q0"] < n) and np.all(g["q1"] < n)
        depth = np.sum(g["op"] == W.OP_U) // n
        assert 10 <= depth <= 40


def test_mixed_circuit_pairs_are_distinct():
    g = W.random_mixed(20, 200, seed=1)
    two = g[g["op"] >= W.OP_CNOT]
    assert np.all(two["q0"] != two["q1"])
    assert 0.25 < len(two) / len(g) < 0.55


def test_wide_bitstrings_round_trip():
    # little-endian words: qubit q is bit q % 64 of word q // 64
    for n in (64, 100, 128, 240):
        z = W.bitstrings_wide(n, 32, seed=n)
        assert z.shape == (32, (n + 63) // 64) and z.dtype == np.uint64
        ints = W.words_to_ints(z)
        assert max(v.bit_length() for v in ints) <= n
        assert np.array_equal(W.ints_to_words(ints, n), z)
    one = W.ints_to_words([1 << 100], 128)
    assert one.tolist() == [[0, 1 << 36]]


def test_block_parts_and_ghz_crossings():
    side = W.block_parts(128, 8)
    assert np.array_equal(np.bincount(side), [16] * 8)
    assert np.array_equal(np.bincount(W.block_parts(10, 3)), [4, 3, 3])
    # the GHZ chain crosses every block boundary once
    assert len(dec.crossing_gates(W.ghz(128), side)) == 7


def test_grid42_cut():
    circ, side = W.grid_circuit(7, 6, 12, seed=7, max_cross=12)
    assert np.array_equal(np.bincount(side), [21, 21])
    assert len(dec.crossing_gates(circ, side)) == 12


def test_grid_diag_closed_form_is_the_oracle_state():
    # the closed form the 48-qubit decomposition test relies on, pinned on a
    # 3x4 grid against the oracle's full state vector and its Eq. (3) sum
    from _closed_forms import diag_closed_form
    from oracle import decomposition as odec
    from oracle import statevector as sv
    circ, side = W.grid_diag_circuit(3, 4, 6, seed=9, max_cross=4)
    n = 12
    assert len(odec.crossing_gates(circ, side)) == 4
    full = sv.run_circuit(n, circ)
    z = np.arange(1 << n, dtype=np.uint64)
    assert np.max(np.abs(diag_closed_form(circ, n, z) - full)) < 1e-14
    zs = [0, 5, 777, (1 << n) - 1]
    ob = odec.branch_amplitudes(n, circ, side, zs)
    assert np.max(np.abs(ob - full[zs])) < 1e-14


def test_grid_diag_circuit_shape():
    # the 48-qubit grid's cut: the same crossing rule as grid_circuit
    circ, side = W.grid_diag_circuit()
    from oracle import decomposition as odec
    assert len(odec.crossing_gates(circ, side)) == 10
    assert np.sum(circ["op"] == W.OP_U) == 48
    assert set(np.unique(circ["op"])) == {W.OP_U, W.OP_T, W.OP_S, W.OP_CZ}
    full_cz = W.grid_circuit(6, 8, 8, seed=5, max_cross=10)[0]
    assert np.array_equal(circ[circ["op"] == W.OP_CZ][["q0", "q1"]], full_cz[full_cz["op"] == W.OP_CZ][["q0", "q1"]])
