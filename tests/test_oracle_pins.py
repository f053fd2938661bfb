"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each expected value is a
literal textbook or paper value, a closed form, an independent construction
(dense brute force, a second decomposition), or an invariant.
"""
import cmath
import math

import numpy as np
import pytest

from oracle import decomposition as dec
from oracle import dense, enc2, observables, statevector as sv
from paper_1912_03243_amd import workloads as W

R2 = 1.0 / math.sqrt(2.0)


# ---- literal textbook actions (Section 2, Eq. (1); Section 4 for CZ) -------

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

@pytest.mark.parametrize(
    "rec, start, expect",
    [
        (W.gate(W.OP_H, 0), 0, {0: R2, 1: R2}),
        (W.gate(W.OP_H, 0), 1, {0: R2, 1: -R2}),
        (W.gate(W.OP_X, 0), 0, {1: 1.0}),
        (W.gate(W.OP_Y, 0), 0, {1: 1j}),
        (W.gate(W.OP_Y, 0), 1, {0: -1j}),
        (W.gate(W.OP_Z, 0), 1, {1: -1.0}),
        (W.gate(W.OP_S, 0), 1, {1: 1j}),
        (W.gate(W.OP_T, 0), 1, {1: cmath.exp(0.25j * math.pi)}),
        (W.gate(W.OP_H, 1), 0, {0: R2, 2: R2}),                 # qubit 1 = bit 1
        (W.gate(W.OP_CNOT, 0, 1), 1, {3: 1.0}),                 # control q0 set: flip q1
        (W.gate(W.OP_CNOT, 0, 1), 2, {2: 1.0}),                 # control clear: nothing
        (W.gate(W.OP_CNOT, 1, 0), 2, {3: 1.0}),
        (W.gate(W.OP_CZ, 0, 1), 3, {3: -1.0}),
        (W.gate(W.OP_CZ, 0, 1), 1, {1: 1.0}),
        (W.gate(W.OP_CP, 1, 0, theta=0.3), 3, {3: cmath.exp(0.3j)}),
        (W.gate(W.OP_U, 1, u=[[0, 1j], [1j, 0]]), 0, {2: 1j}),
    ],
)
def test_literal_gate_actions(rec, start, expect):
    psi = sv.init_state(2, start)
    sv.apply_record(psi, 2, rec[0])
    want = np.zeros(4, dtype=complex)
    for k, v in expect.items():
        want[k] = v
    assert np.max(np.abs(psi - want)) < 1e-15


def test_bell_state():
    psi = sv.run_circuit(2, W.concat(W.gate(W.OP_H, 0), W.gate(W.OP_CNOT, 0, 1)))
    assert np.allclose(psi, [R2, 0, 0, R2], atol=1e-15)


# ---- dense brute force (Section 2: 2^N x 2^N matrix-vector products) -------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_pair_loops_match_dense(n):
    p1 = 1.0 if n == 1 else 0.6
    circ = W.random_mixed(n, 60, seed=100 + n, p1=p1)
    a = sv.run_circuit(n, circ)
    b = dense.run_dense(n, circ)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("targets", [(0,), (4,), (1, 3), (3, 1), (0, 2, 5), (5, 0, 3, 1)])
def test_apply_matrix_matches_dense(targets):
    n = 6
    rng = np.random.default_rng(3)
    k = len(targets)
    z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    m, _ = np.linalg.qr(z)
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    a = psi0.copy()
    sv.apply_matrix(a, n, targets, m)
    b = dense.embed(n, targets, m) @ psi0
    assert np.max(np.abs(a - b)) < 1e-13


def test_controlled_matches_dense_both_orders():
    n = 5
    rng = np.random.default_rng(11)
    u, _ = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
    psi0 = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    for c, t in [(0, 4), (4, 0), (2, 3), (3, 1)]:
        a = psi0.copy()
        sv.apply_controlled(a, n, c, t, u)
        cu = np.eye(4, dtype=complex)
        cu[np.ix_([1, 3], [1, 3])] = u        # control = index bit 0, target = bit 1
        b = dense.embed(n, (c, t), cu) @ psi0
        assert np.max(np.abs(a - b)) < 1e-13


# ---- invariants ---------------------------------------------------------------
def test_norm_and_inverse_round_trip():
    n = 10
    circ = W.random_mixed(n, 200, seed=5)
    psi = sv.run_circuit(n, circ)
    assert abs(sv.norm(psi) - 1.0) < 1e-13 * len(circ)
    back = sv.run_circuit(n, W.inverse_circuit_records(circ), psi=psi)
    assert abs(back[0] - 1.0) < 1e-12
    assert np.max(np.abs(back[1:])) < 1e-12


def test_norm_is_sum_of_squares():
    psi = np.array([3 + 4j, 0, 1j, -2], dtype=complex)
    assert sv.norm(psi) == 30.0


# ---- known-outcome circuits (Section 3) --------------------------------------
@pytest.mark.parametrize("n", [1, 2, 7, 12])
def test_hadamard_all_uniform_and_expectations(n, golden):
    psi = sv.run_circuit(n, W.hadamard_all(n))
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15
    q = observables.q_expectations(psi, n)
    assert np.allclose(q[:, 0], golden["hadamard_all.Q_x"], atol=1e-14)
    assert np.allclose(q[:, 1], golden["hadamard_all.Q_y"], atol=1e-14)
    assert np.allclose(q[:, 2], golden["hadamard_all.Q_z"], atol=1e-14)


@pytest.mark.parametrize("n", [2, 3, 9, 14])
def test_ghz(n, golden):
    psi = sv.run_circuit(n, W.ghz(n))
    want = np.zeros(1 << n, dtype=complex)
    want[0] = golden["ghz.amp_all_zero"]
    want[-1] = golden["ghz.amp_all_one"]
    assert np.max(np.abs(psi - want)) < 1e-15


def test_pauli_expectations_single_qubit_states():
    # |0>: <sz> = 1;  |+>: <sx> = 1;  (|0> + i|1>)/sqrt2: <sy> = 1
    for vec, alpha in [([1, 0], "z"), ([R2, R2], "x"), ([R2, 1j * R2], "y")]:
        psi = np.array(vec, dtype=complex)
        assert abs(observables.pauli_expectation(psi, 1, 0, alpha) - 1.0) < 1e-15


@pytest.mark.parametrize("n, x", [(3, 0), (3, 5), (6, 1), (6, 37), (9, 300)])
def test_qft_of_basis_state(n, x):
    psi = sv.run_circuit(n, W.concat(W.prepare_basis(n, x), W.qft(n)))
    y = np.arange(1 << n)
    want = np.exp(2j * np.pi * x * y / (1 << n)) / 2.0 ** (n / 2)
    assert np.max(np.abs(psi - want)) < 1e-13


def test_swap_network_matches_permutation():
    n = 5
    rng = np.random.default_rng(2)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    a, b = 1, 4
    swapped = psi.copy()
    for c, t in [(a, b), (b, a), (a, b)]:
        sv.apply_controlled(swapped, n, c, t, np.array([[0, 1], [1, 0]], dtype=complex))
    perm = list(range(n))
    perm[a], perm[b] = b, a
    assert np.max(np.abs(sv.permute_qubits(psi, n, perm) - swapped)) < 1e-15


# ---- Eq. (2): CZ decomposition ---------------------------------------------------
@pytest.mark.parametrize("x", dec.ROOTS)
def test_eq2_reproduces_cz_for_every_root(x, golden):
    assert abs(cmath.cos(2 * x) - complex(*golden["eq2.cos2x"])) < 1e-15
    assert np.max(np.abs(dec.eq2_sum(x) - np.diag(golden["cz.diag"]))) < 1e-15


def test_projector_identity_is_cz():
    p0, p1 = np.diag([1.0, 0.0]), np.diag([0.0, 1.0])
    i2, z = np.eye(2), np.diag([1.0, -1.0])
    m = np.kron(i2, p0) + np.kron(z, p1)          # qubit i = index bit 0
    assert np.array_equal(m, np.diag([1.0, 1.0, 1.0, -1.0]))


def test_branch_factor_magnitudes():
    # |e^{i(xs - pi/4)}| = e^{-s Im x}: 1.5538... and 0.6436... for the chosen root
    d = dec.branch_diag(1)
    assert abs(abs(d[0, 0]) - math.exp(0.5 * math.asinh(1.0))) < 1e-15
    assert abs(abs(d[1, 1]) - math.exp(-0.5 * math.asinh(1.0))) < 1e-15


# ---- Eq. (3): branch sum equals the full-state amplitude ---------------------------
@pytest.mark.parametrize("rows, cols, depth, seed", [(2, 4, 4, 3), (4, 4, 8, 9), (2, 6, 6, 1)])
def test_eq3_matches_full_state(rows, cols, depth, seed):
    circ, side = W.grid_circuit(rows, cols, depth, seed, max_cross=None)
    n = rows * cols
    full = sv.run_circuit(n, circ)
    zs = np.arange(1 << n) if n <= 8 else np.random.default_rng(seed).integers(0, 1 << n, 64)
    got = dec.branch_amplitudes(n, circ, side, zs)
    assert len(dec.crossing_gates(circ, side)) >= 1
    assert np.max(np.abs(got - full[zs])) < 1e-12


@pytest.mark.parametrize("nparts, seed", [(3, 5), (4, 6)])
def test_eq3_more_parts_matches_full_state(nparts, seed):
    # Section 4 allows any partition into mutually exclusive subsets: three
    # or four parts of three qubits with 5 crossing CZs, against the full
    # state vector
    n, side, circ = parts_circuit(nparts, seed)
    full = sv.run_circuit(n, circ)
    zs = np.random.default_rng(seed).integers(0, 1 << n, 48)
    got = dec.branch_amplitudes(n, circ, side, zs)
    assert int(side.max()) + 1 == nparts
    assert np.max(np.abs(got - full[zs])) < 1e-12


@pytest.mark.parametrize("x", dec.ROOTS)
def test_eq3_independent_of_root_and_matches_projectors(x):
    circ, side = W.grid_circuit(2, 4, 6, 4, max_cross=None)
    zs = np.arange(256)
    a = dec.branch_amplitudes(8, circ, side, zs, x=x)
    b = dec.projector_amplitudes(8, circ, side, zs)
    assert np.max(np.abs(a - b)) < 1e-12


def test_ghz_via_decomposition(golden):
    # GHZ chain cut in the middle: one crossing CZ after rewriting the crossing
    # CNOT as H_t CZ H_t (textbook identity, Section 4 uses CZ for every
    # entangling gate).
    n = 10
    recs = [W.gate(W.OP_H, 0)]
    for i in range(n - 1):
        if i == n // 2 - 1:
            recs += [W.gate(W.OP_H, i + 1), W.gate(W.OP_CZ, i, i + 1), W.gate(W.OP_H, i + 1)]
        else:
            recs.append(W.gate(W.OP_CNOT, i, i + 1))
    circ = W.concat(*recs)
    side = np.array([0] * (n // 2) + [1] * (n // 2))
    got = dec.branch_amplitudes(n, circ, side, [0, (1 << n) - 1, 5])
    assert abs(got[0] - golden["ghz.amp_all_zero"]) < 1e-15
    assert abs(got[1] - golden["ghz.amp_all_one"]) < 1e-15
    assert abs(got[2]) < 1e-15


@pytest.mark.parametrize("seed", [11, 12])
def test_eq3_crossing_cnots_match_full_state_and_projectors(seed):
    # a crossing CNOT is its CZ between Hadamards on the target; the
    # projector sum uses |1><1| (x) X directly, with no Hadamards
    n, side, circ = W.cnot_cut_circuit(seed)
    assert len(dec.crossing_gates(circ, side)) == 5
    full = sv.run_circuit(n, circ)
    zs = np.arange(1 << n)
    a = dec.branch_amplitudes(n, circ, side, zs)
    b = dec.projector_amplitudes(n, circ, side, zs)
    assert np.max(np.abs(a - full)) < 1e-12
    assert np.max(np.abs(b - full)) < 1e-12


def test_ghz128_paper_values(golden):
    # Section 4's scaling run: the GHZ circuit on 128 qubits, here in eight
    # parts of 16 (7 crossing CNOTs); the coefficients of |0...0> and
    # |1...1> are 1/sqrt(2).  Every other coefficient is zero: exactly when a
    # part's bits are mixed (each part state lives on its all-0 and all-1
    # strings), up to rounding when every part is uniform but the parts differ
    # (the branch sum cancels).
    n = 128
    side = W.block_parts(n, 8)
    ones = (1 << n) - 1
    uniform_mixed = [sum(((1 << 16) - 1) << (16 * p) for p in range(8) if (m >> p) & 1)
                     for m in (0b00000001, 0b10110010, 0b01111111)]
    rand = W.words_to_ints(W.bitstrings_wide(n, 3, 7))
    got = dec.branch_amplitudes(n, W.ghz(n), side, [0, ones] + uniform_mixed + rand)
    assert abs(got[0] - golden["ghz.amp_all_zero"]) < 1e-14
    assert abs(got[1] - golden["ghz.amp_all_one"]) < 1e-14
    assert np.max(np.abs(got[2:5])) < 1e-14
    assert np.all(got[5:] == 0)


def test_ghz_then_haar_layer_closed_form():
    # U_0 (x) ... (x) U_{n-1} applied to (|0...0> + |1...1>)/sqrt(2) has the
    # coefficient (prod_q U_q[z_q, 0] + prod_q U_q[z_q, 1]) / sqrt(2) at z: a
    # closed form for any z, here at n = 96 in six parts (5 crossing CNOTs)
    n = 96
    layer = W.haar_layer(n, 21)
    circ = W.concat(W.ghz(n), layer)
    side = W.block_parts(n, 6)
    zs = W.words_to_ints(W.bitstrings_wide(n, 6, 22)) + [0, (1 << n) - 1]
    got = dec.branch_amplitudes(n, circ, side, zs)
    u = layer["u"].reshape(n, 2, 2, 2)
    u = u[..., 0] + 1j * u[..., 1]
    for k, z in enumerate(zs):
        bits = [(z >> q) & 1 for q in range(n)]
        a0 = np.prod([u[q, bits[q], 0] for q in range(n)])
        a1 = np.prod([u[q, bits[q], 1] for q in range(n)])
        want = (a0 + a1) / math.sqrt(2.0)
        assert abs(got[k] - want) <= 1e-12 * abs(want)


# ---- reference two-byte codec -------------------------------------------------------
def test_enc2_special_blocks():
    B = 2
    amps = np.array([0, 0, 0, 0,                      # all-zero block
                     0, 0.5j, 0, 0,                   # one non-zero component
                     -3.0, 0.25, 1e-39, 0,            # max on a negative real part
                     2.0 ** -110, 0, 0, 0], dtype=complex)   # below 2^-100: stored as zero
    codes, scales = enc2.encode(amps, B)
    assert scales.tolist() == [0.0, 0.5, 3.0, 0.0]
    assert codes[:4].tolist() == [[0, 0]] * 4
    assert codes[4:8].tolist() == [[0, 0], [0, 127], [0, 0], [0, 0]]
    # 0.25 * fl(127/3) = 10.583... -> 11;  1e-39 -> 0
    assert codes[8:12].tolist() == [[-127, 0], [11, 0], [0, 0], [0, 0]]
    assert codes[12:].tolist() == [[0, 0]] * 4


def test_enc2_round_half_to_even():
    # scale 127 gives r = 1 exactly, so the products are the inputs themselves
    amps = np.array([127.0, 2.5, 3.5, -2.5 + 0.5j], dtype=complex)
    codes, scales = enc2.encode(amps, 2)
    assert scales[0] == 127.0
    assert codes.tolist() == [[127, 0], [2, 0], [4, 0], [-2, 0]]


def test_enc2_exact_for_uniform_and_ghz_states(golden):
    for n in (4, 7, 10):
        psi = sv.run_circuit(n, W.hadamard_all(n))
        codes, scales = enc2.encode(psi, 3)
        assert np.all(codes[:, 0] == 127) and np.all(codes[:, 1] == 0)
        dec_ = enc2.decode(codes, scales, 3)
        assert np.all(dec_ == np.complex64(2.0 ** (-n / 2)))
    g = sv.run_circuit(6, W.ghz(6))
    codes, scales = enc2.encode(g, 6)
    d = enc2.decode(codes, scales, 6)
    assert d[0] == d[-1] == np.float32(golden["ghz.amp_all_zero"])


def test_enc2_error_bound_and_reencode():
    rng = np.random.default_rng(8)
    B = 5
    amps = (rng.standard_normal(1 << 12) + 1j * rng.standard_normal(1 << 12)) * 1e-3
    codes, scales = enc2.encode(amps, B)
    back = enc2.decode(codes, scales, B)
    s = np.repeat(scales, 1 << B)
    x32 = amps.astype(np.complex64)
    err = np.maximum(np.abs(back.real - x32.real), np.abs(back.imag - x32.imag))
    assert np.all(err <= s / 254.0 * (1 + 1e-5))
    # half a quantisation step is also reached (the bound is tight)
    assert np.max(err / s) > 0.45 / 127
    codes2, scales2 = enc2.encode(back, B)
    assert np.array_equal(codes2, codes)


def test_enc2_ragged_tail():
    amps = np.arange(1, 11) * (0.1 + 0.05j)
    codes, scales = enc2.encode(amps, 2)
    assert scales.size == 3
    assert codes[-1, 0] == 127 and codes[-2, 0] == round(9 * 127 / 10)
