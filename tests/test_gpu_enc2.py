"""GPU checks of the two-byte amplitude form inside tile passes.

* A pass whose gates are exact in FP32 (X, Y, Z, S, CNOT, CZ: entries 0,
  +-1, +-i) only permutes and re-signs the decoded amplitudes, so the codes
  and scales it writes must equal the reference codec's encoding of those
  values bit for bit (every pass re-encodes, so the reference re-encodes
  after every pass too).
* After passes with arbitrary gates every block must be a valid code: a zero
  block has scale 0 and zero codes; otherwise some component codes to +-127,
  and re-encoding the decoded block gives the same codes (and the decoded
  block maximum as its scale).
* The error against the FP64 oracle must stay within the quantisation
  model: each re-encode rounds every component to a step d = s / 127 of its
  block (s = the block maximum), an error uniform in [-d/2, d/2] with
  variance d^2 / 12, independent from pass to pass.

Every case prints its name before the GPU work so a failing run names it.
"""
import math

import numpy as np
import pytest

from oracle import enc2 as oenc2
from oracle import statevector as sv
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


def exact_circuit(n, count, seed):
    """Gates whose matrices hold only 0, +-1 and +-i."""
    rng = np.random.default_rng(seed)
    ops = [W.OP_X, W.OP_Y, W.OP_Z, W.OP_S, W.OP_CNOT, W.OP_CZ]
    recs = []
    for _ in range(count):
        op = int(rng.choice(ops))
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        recs.append(W.gate(op, a, b if op in (W.OP_CNOT, W.OP_CZ) else -1))
    return W.concat(*recs)


def noisy_state(J, s, n):
    """Fills the two-byte state s with spread amplitudes (a few brick layers)
    and returns its decoded values as complex128 (exact)."""
    s.init(0)
    s.run(W.layered_brick(n, 3, seed=80 + n), mode="tile", relabel=-1)
    codes, scales = s.raw_codes()
    return oenc2.decode(codes, scales, s.block_bits).astype(np.complex128)


@pytest.mark.parametrize("n, B", [(13, 8), (12, 5)])
def test_one_pass_reencode_is_the_reference_codec(J, n, B):
    # the whole state is one tile: all 40 exact gates in one pass, one re-encode
    announce("enc2-exact-one-pass", n, B)
    circ = exact_circuit(n, 40, seed=81 + n)
    with J.State(n, "enc2", block_bits=B) as s:
        x0 = noisy_state(J, s, n)
        o = s.run(circ, mode="tile", relabel=-1, pass_gates=-1)
        codes1, scales1 = s.raw_codes()
    assert o.passes == 1
    # exact in FP64 and representable in FP32: the values the pass encodes
    phi = sv.run_circuit(n, circ, psi=x0).astype(np.complex64)
    want_codes, want_scales = oenc2.encode(phi, B)
    assert np.array_equal(scales1, want_scales)
    assert np.array_equal(codes1, want_codes)


@pytest.mark.parametrize("n, B", [(16, 8), (15, 10)])
def test_every_pass_reencode_is_the_reference_codec(J, n, B):
    # one gate per run, so one pass (one decode, exact gate, re-encode) per
    # gate; the reference re-encodes after every gate the same way
    announce("enc2-exact-per-pass", n, B)
    circ = exact_circuit(n, 30, seed=82 + n)
    with J.State(n, "enc2", block_bits=B) as s:
        x = noisy_state(J, s, n)
        for k in range(len(circ)):
            o = s.run(circ[k:k + 1], mode="tile", relabel=-1)
            assert o.passes == 1
            x = sv.run_circuit(n, circ[k:k + 1], psi=x)
            codes, scales = oenc2.encode(x.astype(np.complex64), B)
            x = oenc2.decode(codes, scales, B).astype(np.complex128)
        codes1, scales1 = s.raw_codes()
    assert np.array_equal(scales1, scales)
    assert np.array_equal(codes1, codes)


@pytest.mark.parametrize("n, B, relabel", [(16, 8, 0), (18, 6, 0), (17, 12, -1)])
def test_codes_valid_after_passes(J, n, B, relabel):
    announce("enc2-valid", n, B, relabel)
    circ = W.concat(W.layered_brick(n, 6, seed=90 + n), W.random_mixed(n, 80, seed=91 + n))
    with J.State(n, "enc2", block_bits=B) as s:
        s.init(0)
        s.run(circ, mode="tile", relabel=relabel)
        codes, scales = s.raw_codes()
    bs = 1 << B
    blocks = codes.reshape(-1, bs * 2).astype(np.int32)
    zero = scales == 0
    assert np.all(blocks[zero] == 0)
    assert np.all(np.abs(blocks).max(axis=1)[~zero] == 127)
    assert np.all(np.abs(blocks) <= 127)
    dec = oenc2.decode(codes, scales, B)
    c2, s2 = oenc2.encode(dec, B)
    assert np.array_equal(c2, codes)
    want = (np.float32(127) * (scales / np.float32(127)).astype(np.float32)).astype(np.float32)
    assert np.array_equal(s2, want)


@pytest.mark.parametrize("n, B", [(14, 8), (14, 4)])
def test_error_within_quantisation_model(J, n, B):
    # one gate per run, so every run is one pass with one re-encode; the
    # scales after each pass give that re-encode's error variance
    circ = W.concat(W.layered_brick(n, 6, seed=95 + n), W.random_mixed(n, 40, seed=96 + n))
    announce("enc2-error-model", n, B, len(circ))
    var = 0.0
    passes = 0
    with J.State(n, "enc2", block_bits=B) as s:
        s.init(0)
        for k in range(len(circ)):
            o = s.run(circ[k:k + 1], mode="tile", relabel=-1)
            passes += o.passes
            _, scales = s.raw_codes()
            d = scales.astype(np.float64) / 127.0
            var += o.passes * float(np.sum(2 * (1 << B) * d * d / 12.0))
        got = s.state_vector()
    phi = sv.run_circuit(n, circ)
    err = float(np.linalg.norm(got - phi))
    expect = math.sqrt(var)
    fid = abs(np.vdot(phi, got)) ** 2 / (np.vdot(phi, phi).real * np.vdot(got, got).real)
    print(f"enc2 n={n} B={B}: {passes} passes, |err| = {err:.3e}, model rms {expect:.3e}, "
          f"ratio {err / expect:.2f}, 1 - fidelity {1 - fid:.3e}, "
          f"max|err|/max|phi| {np.abs(got - phi).max() / np.abs(phi).max():.3e}", flush=True)
    # FP32 gate arithmetic adds about 2^-24 per operation: far below the steps
    assert err <= 3.0 * expect + 1e-5
