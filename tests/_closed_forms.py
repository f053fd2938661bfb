"""Closed forms used as independent pins (test infrastructure)."""
import numpy as np

from paper_1912_03243_amd import workloads as W


def diag_closed_form(gates, n, zs):
    """<z|C|0> for a Haar layer followed by diagonal gates only (T, S, CZ):
    prod_q U_q[z_q, 0] times the phases of the diagonal gates at z."""
    z = np.asarray(zs, dtype=np.uint64)
    bits = ((z[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.int64)
    haar = gates[gates["op"] == W.OP_U]
    assert np.array_equal(haar["q0"], np.arange(n))
    u = haar["u"].reshape(n, 2, 2, 2)
    u = u[..., 0] + 1j * u[..., 1]
    amp = np.prod(u[np.arange(n)[None, :], bits, 0], axis=1)
    rest = gates[len(haar):]
    assert not np.any(rest["op"] == W.OP_U)
    eighths = np.zeros(len(z), dtype=np.int64)  # phase in units of pi/4
    for rec in rest:
        op, a, b = int(rec["op"]), int(rec["q0"]), int(rec["q1"])
        if op == W.OP_T:
            eighths += bits[:, a]
        elif op == W.OP_S:
            eighths += 2 * bits[:, a]
        elif op == W.OP_CZ:
            eighths += 4 * bits[:, a] * bits[:, b]
        else:
            raise AssertionError(f"unexpected op {op}")
    return amp * np.exp(0.25j * np.pi * (eighths % 8))
