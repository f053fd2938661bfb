"""GPU parity: gate kernels, planner modes and read-out against the oracle.

Every case prints its name before the GPU work so a failing run names it.
"""
import math

import numpy as np
import pytest

from _parity import assert_c128, assert_c64, assert_dtype, bf16_bound, bf16x3_bound, rel_l2
from oracle import enc2 as oenc2
from oracle import observables, statevector as sv
from paper_1912_03243_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_03243_amd import juqcs
    return juqcs


def announce(*what):
    print("CASE", *what, flush=True)


def random_unitary(k, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
    q, r = np.linalg.qr(z)
    return q * (np.diagonal(r) / np.abs(np.diagonal(r)))[None, :]


# ---- init / norm / amplitudes -------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
@pytest.mark.parametrize("idx", [0, 5, 1023])
def test_init_norm_amplitudes(J, dtype, idx):
    announce("init", dtype, idx)
    n = 10
    with J.State(n, dtype) as s:
        s.init(idx)
        amps = s.amplitudes(np.arange(1 << n))
        want = np.zeros(1 << n, dtype=complex)
        want[idx] = 1.0
        assert np.array_equal(amps, want)
        assert s.norm() == 1.0


# ---- plain per-gate kernels -------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 13])
def test_plain_random_circuit(J, dtype, n):
    announce("plain", dtype, n)
    circ = W.random_mixed(n, 120, seed=40 + n, p1=1.0 if n == 1 else 0.6)
    with J.State(n, dtype) as s:
        s.init(0)
        o = s.run(circ, mode="plain")
        assert o.gates == len(circ)
        got = s.state_vector()
    assert_dtype(dtype, got, sv.run_circuit(n, circ))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 22])
def test_every_target_and_control_bit(J, dtype, n):
    # every target bit with a control below and above the run width of the
    # per-gate kernels (64 C128 / 128 C64 amplitudes) at n = 22, whose runs
    # split into low bits (partners across lanes) and high bits (pairs of runs)
    rng = np.random.default_rng(7)
    prefix = W.layered_brick(n, 1, seed=3)
    base = sv.run_circuit(n, prefix, basis_index=3)
    for t in range(n):
        other = int((t + 1 + rng.integers(0, n - 1)) % n)
        recs = [W.gate(W.OP_U, t, u=random_unitary(1, t)),
                W.gate(W.OP_CNOT, t, other), W.gate(W.OP_CNOT, other, t),
                W.gate(W.OP_CZ, t, other), W.gate(W.OP_CP, other, t, theta=0.3 + t),
                W.gate(W.OP_T, t), W.gate(W.OP_Y, t), W.gate(W.OP_H, t)]
        circ = W.concat(*recs)
        announce("target", dtype, n, t, other)
        with J.State(n, dtype) as s:
            s.init(3)
            s.run(W.concat(prefix, circ), mode="plain")
            got = s.state_vector()
        assert_dtype(dtype, got, sv.run_circuit(n, circ, psi=base.copy()))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_calls_match_oracle(J, dtype):
    n = 9
    rng = np.random.default_rng(1)
    circ = W.layered_brick(n, 2, seed=8)
    phi = sv.run_circuit(n, circ)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(circ, mode="plain")
        for step in range(12):
            a, b = rng.choice(n, 2, replace=False)
            u = random_unitary(1, 100 + step)
            m4 = random_unitary(2, 200 + step)
            announce("apply", dtype, step, a, b)
            s.apply_1q(int(a), u)
            sv.apply_1q(phi, n, int(a), u)
            s.apply_controlled(int(a), int(b), u)
            sv.apply_controlled(phi, n, int(a), int(b), u)
            s.apply_2q(int(a), int(b), m4)
            sv.apply_matrix(phi, n, (int(a), int(b)), m4)
            s.apply_1q(int(b), np.diag([1.0, np.exp(0.7j)]))       # diagonal fast path
            sv.apply_1q(phi, n, int(b), np.diag([1.0, np.exp(0.7j)]))
            s.apply_1q(int(a), np.diag([np.exp(0.2j), np.exp(-0.4j)]))
            sv.apply_1q(phi, n, int(a), np.diag([np.exp(0.2j), np.exp(-0.4j)]))
        got = s.state_vector()
    assert_dtype(dtype, got, phi)


# ---- tile passes -------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n, tile_bits, low_bits", [
    (3, 0, 0), (5, 0, 0), (12, 0, 0), (13, 0, 0), (16, 10, 4), (16, 12, 6), (18, 0, 0),
    (20, 13, 5)])
def test_tile_random_circuit(J, dtype, n, tile_bits, low_bits):
    if dtype == "c128" and tile_bits > 13:
        pytest.skip("C128 tiles hold at most 2^13 amplitudes")
    announce("tile", dtype, n, tile_bits, low_bits)
    circ = W.random_mixed(n, 160, seed=60 + n)
    with J.State(n, dtype) as s:
        s.init(1)
        o = s.run(circ, mode="tile", tile_bits=tile_bits, low_bits=low_bits)
        got = s.state_vector()
    assert o.passes >= 1
    assert_dtype(dtype, got, sv.run_circuit(n, circ, basis_index=1))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tile_brick_circuit_fewer_passes(J, dtype):
    n = 20
    circ = W.layered_brick(n, 10, seed=2)
    announce("tile-brick", dtype)
    with J.State(n, dtype) as s:
        s.init(0)
        o = s.run(circ, mode="tile")
        got = s.state_vector()
    assert o.passes < len(circ) / 5
    assert_dtype(dtype, got, sv.run_circuit(n, circ))


def monomial_circuit(n, count, seed):
    # only permutations with phases (X, Y, Z, S, T, CNOT, CZ, CP) after a
    # layer of H: the in-pass fusion turns them into monomial ops
    rng = np.random.default_rng(seed)
    recs = [W.gate(W.OP_H, q) for q in range(n)]
    for _ in range(count):
        op = int(rng.choice([W.OP_X, W.OP_Y, W.OP_Z, W.OP_S, W.OP_T, W.OP_CNOT, W.OP_CZ, W.OP_CP]))
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        recs.append(W.gate(op, a, b if op >= W.OP_CNOT else -1, theta=float(rng.uniform(0, 6.3))))
    return W.concat(*recs)


@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
@pytest.mark.parametrize("n", [9, 16])
def test_tile_monomial_ops(J, dtype, n):
    announce("tile-monomial", dtype, n)
    circ = monomial_circuit(n, 150, seed=40 + n)
    with J.State(n, dtype) as s:
        s.init(0)
        o = s.run(circ, mode="tile")
        got = s.state_vector()
    phi = sv.run_circuit(n, circ)
    if dtype == "enc2":
        assert rel_l2(got, phi) < 0.02 * math.sqrt(o.passes + 1)
    else:
        assert_dtype(dtype, got, phi)


@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
@pytest.mark.parametrize("pass_gates", [-1, 0, 7, 40])
def test_tile_pass_gate_cap(J, dtype, pass_gates):
    # a cap only moves gates to later passes (and splits clusters): same state
    n = 16
    circ = W.layered_brick(n, 8, seed=4)
    announce("tile-cap", dtype, pass_gates)
    with J.State(n, dtype) as s:
        s.init(0)
        o = s.run(circ, mode="tile", pass_gates=pass_gates)
        got = s.state_vector()
    phi = sv.run_circuit(n, circ)
    if pass_gates == 7:
        assert o.passes >= len(circ) / 7
    if dtype == "enc2":
        assert rel_l2(got, phi) < 0.02 * math.sqrt(o.passes + 1)
    else:
        assert_dtype(dtype, got, phi)


# ---- relabeling: passes hand the low physical bits to other qubits ---------------
RELABEL_CASES = [  # (n, tile_bits, low_bits, fuse_k): kernel exercised
    (20, 0, 0, 0),    # default tile: pipelined 2^13 kernel
    (18, 12, 5, 0),   # pipelined 2^12 kernel (two workgroups per CU)
    (18, 11, 4, 0),   # pipelined 2^11 kernel
    (16, 10, 3, 0),   # generic kernel (tile below the pipelined sizes)
    (18, 12, 4, 4),   # generic kernel (16x16 ops)
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", RELABEL_CASES)
def test_tile_relabel(J, dtype, case):
    n, tb, lb, fk = case
    circ = W.concat(W.layered_brick(n, 12, seed=60 + n), W.random_mixed(n, 80, seed=61 + n))
    announce("tile-relabel", dtype, case)
    z = np.arange(0, 1 << n, 997, dtype=np.uint64)
    with J.State(n, dtype) as s:
        s.init(3)
        off = s.run(circ, mode="tile", tile_bits=tb, low_bits=lb, fuse_k=fk, relabel=-1)
        assert s.layout() == list(range(n))
        s.init(3)
        on = s.run(circ, mode="tile", tile_bits=tb, low_bits=lb, fuse_k=fk, relabel=1)
        layout = s.layout()
        amps = s.amplitudes(z)            # read through the moved layout
        ex = s.expectations()
        got = s.state_vector()            # read through the layout
        assert s.layout() == layout
        s.canonicalize()
        assert s.layout() == list(range(n))
        got2 = s.state_vector()
    phi = sv.run_circuit(n, circ, basis_index=3)
    assert_dtype(dtype, got2, phi)
    assert sorted(layout) == list(range(n))
    assert layout != list(range(n)), "brick circuit on a partial tile: relabeling expected"
    assert on.passes <= off.passes
    assert_dtype(dtype, got, phi)
    assert_dtype(dtype, amps, phi[z.astype(np.int64)])
    tol = 1e-11 if dtype == "c128" else 2e-5
    assert np.max(np.abs(ex - observables.q_expectations(phi, n))) < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tile_relabel_runs_chain(J, dtype):
    # a run starts from the layout the previous one left, also after permute()
    n = 19
    a = W.layered_brick(n, 10, seed=71)
    b = W.random_mixed(n, 150, seed=72)
    c = W.layered_brick(n, 6, seed=73)
    perm = np.random.default_rng(74).permutation(n)
    announce("tile-relabel-chain", dtype)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(a, mode="tile", relabel=1)
        s.run(b, mode="tile", relabel=1)
        s.permute(perm)
        s.run(c, mode="tile", relabel=1)
        s.run(W.ghz(n)[:3], mode="plain")
        got = s.state_vector()
    phi = sv.run_circuit(n, W.concat(a, b, c, W.ghz(n)[:3]))
    assert_dtype(dtype, got, phi)


def test_tile_relabel_rejects_bad_value(J):
    with J.State(8, "c128") as s:
        with pytest.raises(J.JuqcsError) as e:
            s.run(W.layered_brick(8, 2, seed=1), mode="tile", relabel=2)
    assert e.value.status == J.ERR_ARG


@pytest.mark.parametrize("case", [(20, 0, 0), (18, 12, 8)])
def test_tile_relabel_enc2(J, case):
    # two-byte tiles re-encode their blocks in the relabeled order
    n, tb, lb = case
    circ = W.concat(W.layered_brick(n, 10, seed=75 + n), W.random_mixed(n, 60, seed=76 + n))
    announce("tile-relabel-enc2", case)
    z = np.arange(0, 1 << n, 1001, dtype=np.uint64)
    with J.State(n, "enc2") as s:
        s.init(0)
        off = s.run(circ, mode="tile", tile_bits=tb, low_bits=lb, relabel=-1)
        assert s.layout() == list(range(n))
        ref = s.state_vector()
        s.init(0)
        on = s.run(circ, mode="tile", tile_bits=tb, low_bits=lb, relabel=1)
        layout = s.layout()
        amps = s.amplitudes(z)
        ex = s.expectations()
        got = s.state_vector()
    phi = sv.run_circuit(n, circ)
    assert layout != list(range(n))
    assert on.passes <= off.passes
    tol = 0.02 * math.sqrt(on.passes + 1)
    assert rel_l2(got, phi) < tol and rel_l2(ref, phi) < 0.02 * math.sqrt(off.passes + 1)
    assert rel_l2(amps, phi[z.astype(np.int64)]) < 3 * tol
    assert np.max(np.abs(ex - observables.q_expectations(phi, n))) < 3 * tol


def test_tile_pass_gate_cap_rejects_bad_value(J):
    with J.State(8, "c128") as s:
        with pytest.raises(J.JuqcsError) as e:
            s.run(W.layered_brick(8, 2, seed=1), mode="tile", pass_gates=-2)
    assert e.value.status == J.ERR_ARG


# ---- fused k-qubit blocks on the matrix cores --------------------------------------
@pytest.mark.parametrize("dtype, mode", [("c128", "fp64"), ("c64", "fp32"), ("c64", "bf16x3"),
                                         ("c64", "bf16")])
@pytest.mark.parametrize("targets", [(0,), (3, 1), (0, 1, 2), (9, 2, 5, 0), (1, 3, 5, 7, 9),
                                     (10, 0, 4, 8, 2, 6)])
def test_apply_fused_k(J, dtype, mode, targets):
    n = 11
    announce("fused", dtype, mode, targets)
    circ = W.layered_brick(n, 2, seed=5)
    m = random_unitary(len(targets), len(targets))
    phi = sv.run_circuit(n, circ)
    sv.apply_matrix(phi, n, targets, m)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(circ, mode="plain")
        s.apply_fused(targets, m, mode)
        got = s.state_vector()
    if mode == "bf16":
        assert rel_l2(got, phi) <= bf16_bound(1)
    elif mode == "bf16x3":
        assert rel_l2(got, phi) <= bf16x3_bound(1)
    else:
        assert_dtype(dtype, got, phi)


@pytest.mark.parametrize("dtype, mma", [("c128", "fp64"), ("c64", "fp32"), ("c64", "bf16")])
@pytest.mark.parametrize("k", [2, 4, 5, 6])
def test_fused_plan(J, dtype, mma, k):
    n = 14
    announce("fused-plan", dtype, mma, k)
    circ = W.layered_brick(n, 6, seed=11)
    with J.State(n, dtype) as s:
        s.init(0)
        o = s.run(circ, mode="fused", fuse_k=k, mma=mma)
        got = s.state_vector()
    phi = sv.run_circuit(n, circ)
    assert o.passes < len(circ)
    if mma == "bf16":
        assert rel_l2(got, phi) <= bf16_bound(o.passes)
    else:
        assert_dtype(dtype, got, phi)


# ---- layout ------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
def test_permute_and_canonicalize(J, dtype):
    n = 12
    announce("permute", dtype)
    a = W.layered_brick(n, 2, seed=21)
    b = W.random_mixed(n, 60, seed=22)
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(a)
        s.permute(perm)
        assert s.layout() == list(perm)
        s.run(b)
        z = np.arange(0, 1 << n, 7, dtype=np.uint64)
        amps = s.amplitudes(z)
        got = s.state_vector()
        s.canonicalize()
        assert s.layout() == list(range(n))
        got2 = s.state_vector()
    phi = sv.run_circuit(n, W.concat(a, b))
    if dtype == "enc2":
        assert rel_l2(got2, phi) < 0.1
    else:
        assert_dtype(dtype, got2, phi)
    if dtype == "enc2":
        assert rel_l2(got, phi) < 0.1
    else:
        assert_dtype(dtype, got, phi)
        assert_dtype(dtype, amps, phi[z.astype(np.int64)])


# ---- autotuner ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
def test_autotune_picks_and_auto_mode_uses_it(J, dtype, tmp_path):
    n = 16
    announce("autotune", dtype)
    circ = W.layered_brick(n, 8, seed=31)
    other = W.layered_brick(n, 8, seed=32)          # same structure, other matrices
    J.juqcs_tune_clear()
    with J.State(n, dtype) as s:
        t = s.autotune(circ)
        assert t["mode"] in ("tile", "fused", "plain") and t["trials"] >= 8
        assert t["ms"] <= t["default_ms"]
        s.init(0)
        s.run(other, mode="auto")
        got = s.state_vector()
        path = tmp_path / "tune.json"
        J.juqcs_tune_save(str(path))
        J.juqcs_tune_clear()
        J.juqcs_tune_load(str(path))
        s.init(0)
        s.run(other, mode="auto")
        got2 = s.state_vector()
    J.juqcs_tune_clear()
    phi = sv.run_circuit(n, other)
    if dtype == "enc2":
        assert rel_l2(got, phi) < 0.05 and rel_l2(got2, phi) < 0.05
    else:
        assert_dtype(dtype, got, phi)
        assert np.array_equal(got, got2)


# ---- global factor -------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
def test_global_factor(J, dtype):
    # an FP64 complex factor of the whole state: set by one call, carried by
    # diagonal gates' first entries, applied by every read-out, used to
    # renormalise; the stored amplitudes are never touched for it
    n = 13
    announce("global-factor", dtype)
    circ = W.random_mixed(n, 90, seed=17)
    g = 0.3 - 0.7j
    rz = np.diag([np.exp(-0.45j), np.exp(0.45j)])      # diag(a, b): a goes into the factor
    phi = g * sv.run_circuit(n, circ)
    sv.apply_1q(phi, n, 4, rz)
    sv.apply_1q(phi, n, 0, 1.5 * np.eye(2))              # a scalar: no pass at all
    z = np.arange(0, 1 << n, 37, dtype=np.uint64)
    with J.State(n, dtype) as s:
        s.init(0)
        s.set_global_factor(g)
        s.run(circ, mode="tile")
        s.apply_1q(4, rz)
        s.apply_1q(0, 1.5 * np.eye(2))
        gf = s.global_factor()
        amps = s.amplitudes(z)
        full = s.state_vector()
        nrm = s.norm()
        ex = s.expectations()
        before = s.renormalize()
        nrm1 = s.norm()
        amps1 = s.amplitudes(z)
        s.init(0)
        assert s.global_factor() == 1.0
    assert abs(gf - g * np.exp(-0.45j) * 1.5) < 1e-15
    want_n = sv.norm(phi)
    want_q = observables.q_expectations(phi, n)
    if dtype == "enc2":
        tol = 0.05
        assert rel_l2(full, phi) < tol and rel_l2(amps, phi[z.astype(np.int64)]) < tol
        assert abs(nrm / want_n - 1) < tol and abs(before - nrm) < 1e-15 * nrm
        assert abs(nrm1 - 1) < 1e-12
        assert np.max(np.abs(ex - want_q)) < tol
        return
    assert_dtype(dtype, full, phi)
    assert_dtype(dtype, amps, phi[z.astype(np.int64)])
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(nrm - want_n) < tol * want_n and before == nrm
    assert abs(nrm1 - 1.0) < tol
    assert_dtype(dtype, amps1, phi[z.astype(np.int64)] / math.sqrt(want_n))
    assert np.max(np.abs(ex - want_q)) < tol


# ---- read-out ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_norm_expectations_scale(J, dtype):
    n = 14
    announce("observables", dtype)
    circ = W.random_mixed(n, 100, seed=3)
    phi = sv.run_circuit(n, circ)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(circ)
        n1 = s.norm()
        assert n1 == s.norm()                      # fixed reduction order
        ex = s.expectations()
        s.scale(0.5)
        n2 = s.norm()
    want = observables.q_expectations(phi, n)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert abs(n1 - 1.0) < tol and abs(n2 - 0.25) < tol
    assert np.max(np.abs(ex - want)) < tol


@pytest.mark.parametrize("n, dtype, permute", [
    (22, "c128", False), (22, "c64", False), (22, "enc2", False), (22, "c128", True),
    (22, "c64", True), (3, "c128", False), (7, "c64", False), (9, "enc2", False),
    (19, "c128", False), (21, "enc2", False)])
def test_expectations_multi_pass(J, n, dtype, permute):
    # n = 22 needs three tile geometries (13 low bits, then gathered bits),
    # small n a single partial tile; the reference is the oracle's formula
    # on the state the GPU holds
    announce("expectations", n, dtype, permute)
    circ = W.random_mixed(n, 120, seed=11)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(circ, mode="tile")
        if permute:
            s.permute(list(reversed(range(n))))
        ex = s.expectations()
        psi = s.state_vector()
    assert np.max(np.abs(ex - observables.q_expectations(psi, n))) < 1e-11
    if dtype != "enc2":
        want = observables.q_expectations(sv.run_circuit(n, circ), n)
        assert np.max(np.abs(ex - want)) < (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64", "enc2"])
def test_known_outcome_circuits(J, dtype, golden):
    n = 12
    announce("known", dtype)
    with J.State(n, dtype) as s:
        s.init(0)
        s.run(W.hadamard_all(n))
        ex = s.expectations()
        assert np.allclose(ex[:, 0], golden["hadamard_all.Q_x"], atol=1e-6)
        assert np.allclose(ex[:, 1], golden["hadamard_all.Q_y"], atol=1e-6)
        assert np.allclose(ex[:, 2], golden["hadamard_all.Q_z"], atol=1e-6)
        amp = s.amplitudes(np.arange(1 << n))
        assert np.allclose(amp, 2.0 ** (-n / 2), atol=1e-6, rtol=0)
        s.init(0)
        s.run(W.ghz(n), mode="plain")
        amp = s.amplitudes(np.array([0, (1 << n) - 1, 1, 7]))
    tol = 1e-15 if dtype == "c128" else 1e-7
    assert abs(amp[0] - golden["ghz.amp_all_zero"]) < tol
    assert abs(amp[1] - golden["ghz.amp_all_one"]) < tol
    assert np.all(np.abs(amp[2:]) == 0)


def test_enc2_uniform_state_is_exact(J):
    n = 12
    announce("enc2-uniform")
    with J.State(n, "enc2") as s:
        s.init(0)
        s.run(W.hadamard_all(n))
        codes, scales = s.raw_codes()
        ex = s.expectations()
    # every amplitude is the block maximum: one code value, one common scale
    assert np.all(codes[:, 0] == 127) and np.all(codes[:, 1] == 0)
    assert np.all(scales == scales[0])
    assert abs(scales[0] - 2.0 ** (-n / 2)) <= 2.0 ** (-n / 2) * 1e-6
    assert np.allclose(ex, [[0.0, 0.5, 0.5]] * n, atol=1e-6)


# ---- two-byte codec ----------------------------------------------------------------------
@pytest.mark.parametrize("src", ["c128", "c64"])
@pytest.mark.parametrize("count, B", [(1 << 12, 8), (1000, 5), (4096 + 77, 10), (8, 3)])
def test_codec_bit_exact(J, src, count, B):
    import torch
    announce("codec", src, count, B)
    rng = np.random.default_rng(count + B)
    x = (rng.standard_normal(count) + 1j * rng.standard_normal(count)) * 10.0 ** rng.integers(-8, 2, count)
    bs = 1 << B
    x[:bs] = 0                                       # all-zero block
    if count > 2 * bs:
        x[bs:2 * bs] = 0
        x[bs + 3] = -0.75j                           # single non-zero component
        x[2 * bs: 2 * bs + 4] = [127.0, 2.5, -3.5, 1e-39]   # ties at r = 1, denormal
    if src == "c64":
        x = x.astype(np.complex64)
    want_codes, want_scales = oenc2.encode(x, B)
    dt = torch.float64 if src == "c128" else torch.float32
    xs = torch.from_numpy(np.stack([x.real, x.imag], -1).reshape(-1).astype(
        np.float64 if src == "c128" else np.float32)).to("cuda", dt)
    nblk = (count + bs - 1) // bs
    codes = torch.empty(2 * count, dtype=torch.int8, device="cuda")
    scales = torch.empty(nblk, dtype=torch.float32, device="cuda")
    J.juqcs_encode2(xs, J.DTYPES[src], count, B, codes, scales)
    dec = torch.empty(2 * count, dtype=torch.float32, device="cuda")
    J.juqcs_decode2(codes, scales, count, B, dec, J.C64)
    torch.cuda.synchronize()
    assert np.array_equal(codes.cpu().numpy().reshape(-1, 2), want_codes)
    assert np.array_equal(scales.cpu().numpy(), want_scales)
    d = dec.cpu().numpy()
    want_dec = oenc2.decode(want_codes, want_scales, B)
    assert np.array_equal(d[0::2], want_dec.real) and np.array_equal(d[1::2], want_dec.imag)


# ---- errors reported by the library -------------------------------------------------------
def test_error_paths(J):
    announce("errors")
    with J.State(6, "c128") as s:
        s.init(0)
        with pytest.raises(J.JuqcsError) as e:
            s.apply_1q(6, np.eye(2))
        assert e.value.status == J.ERR_QUBIT
        with pytest.raises(J.JuqcsError) as e:
            s.apply_controlled(2, 2, np.eye(2))
        assert e.value.status == J.ERR_QUBIT
        with pytest.raises(J.JuqcsError) as e:
            s.apply_1q(0, np.array([[np.nan, 0], [0, 1]]))
        assert e.value.status == J.ERR_NUMERIC
        with pytest.raises(J.JuqcsError) as e:
            s.apply_fused([1, 1], np.eye(4))
        assert e.value.status == J.ERR_QUBIT
        with pytest.raises(J.JuqcsError) as e:
            s.apply_fused([1, 2], np.eye(4), "fp32")
        assert e.value.status == J.ERR_DTYPE
        with pytest.raises(J.JuqcsError) as e:
            s.run(W.concat(W.gate(W.OP_CZ, 1, 1)))
        assert e.value.status == J.ERR_QUBIT
        with pytest.raises(J.JuqcsError) as e:
            s.permute([0, 0, 1, 2, 3, 4])
        assert e.value.status == J.ERR_QUBIT
        with pytest.raises(J.JuqcsError) as e:
            s.amplitudes([64])
        assert e.value.status == J.ERR_ARG
        # a non-unitary gate is applied as given; the norm reports it
        s.apply_1q(0, 2.0 * np.eye(2))
        assert s.norm() == 4.0
