"""Comparison helpers and the tolerances of the parity tests.

complex128 paths: max |psi - phi| <= 1e-12 and ||psi - phi|| / ||phi|| <= 1e-12.
complex64 paths (plain, tile and FP32 matrix cores): relative L2 error
and max error relative to max |phi| both <= 1e-5.
BF16 matrix cores: each fused pass rounds the state and the block matrix to
BF16 (unit roundoff 2^-9 = 1.95e-3); the accumulated relative L2 error is
bounded by 4 * 2^-9 * sqrt(passes) (inputs rounded on both operands, about
sqrt(2) per pass, with margin).
BF16x3 (hi*hi + hi*lo + lo*hi): every operand is carried to about 17
significant bits (x - hi - lo <= 2^-18 |x|) and lo*lo is dropped, so the
per-pass relative error is about 2^-17; the bound is 4 * 2^-17 * sqrt(passes).
Two-byte states: each re-encode adds at most half a quantisation step, s/254,
per component (s = block max); for spread states the relative L2 error per
re-encode is about 1/(127*sqrt(12)) * (max/rms) <= 1%, so the test bound is
0.02 * sqrt(re-encodes + 1).
"""
import math

import numpy as np

TOL_C128 = 1e-12
TOL_C64 = 1e-5
BF16_U = 2.0 ** -9


def rel_l2(psi, phi):
    return float(np.linalg.norm(psi - phi) / max(np.linalg.norm(phi), 1e-300))


def assert_c128(psi, phi):
    d = np.abs(psi - phi)
    assert float(d.max()) <= TOL_C128, f"max abs err {d.max():.3e}"
    assert rel_l2(psi, phi) <= TOL_C128, f"rel L2 err {rel_l2(psi, phi):.3e}"


def assert_c64(psi, phi, tol=TOL_C64):
    rel = rel_l2(psi, phi)
    mx = float(np.abs(psi - phi).max() / max(np.abs(phi).max(), 1e-300))
    assert rel <= tol, f"rel L2 err {rel:.3e} > {tol:.1e}"
    assert mx <= tol, f"max rel err {mx:.3e} > {tol:.1e}"


def bf16_bound(passes: int) -> float:
    return 4.0 * BF16_U * math.sqrt(max(passes, 1))


def bf16x3_bound(passes: int) -> float:
    return 4.0 * 2.0 ** -17 * math.sqrt(max(passes, 1))


def enc2_bound(reencodes: int) -> float:
    return 0.02 * math.sqrt(reencodes + 1)


def assert_dtype(dtype, psi, phi):
    if dtype == "c128":
        assert_c128(psi, phi)
    else:
        assert_c64(psi, phi)
