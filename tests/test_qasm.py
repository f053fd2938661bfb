"""Circuit front-end (OpenQASM 2.0 subset) on the CPU: parsed programs give
the gate records, and through the oracle the states, of circuits built by
hand, and every unsupported construct is rejected."""
import cmath
import math

import numpy as np
import pytest

from oracle import statevector as sv
from paper_1912_03243_amd import qasm
from paper_1912_03243_amd import workloads as W


def test_ghz_program_matches_generator():
    n = 6
    prog = "OPENQASM 2.0;\ninclude \"qelib1.inc\";\nqreg q[6];\ncreg c[6];\nh q[0];\n"
    prog += "".join(f"cx q[{i}],q[{i + 1}];\n" for i in range(n - 1))
    m, g = qasm.parse_qasm(prog)
    want = W.ghz(n)
    assert m == n
    assert np.array_equal(g["op"], want["op"]) and np.array_equal(g["q0"], want["q0"])
    assert np.array_equal(g["q1"], want["q1"])
    psi = sv.run_circuit(n, g)
    assert abs(psi[0] - 1 / math.sqrt(2)) < 1e-15 and abs(psi[-1] - 1 / math.sqrt(2)) < 1e-15


def test_rotations_and_phases_against_matrices():
    # each parsed gate against the matrix written out here (textbook forms)
    t, p, l = 0.7, -1.1, 2.3
    prog = f"""OPENQASM 2.0; qreg a[2]; qreg b[1];
    rx({t}) a[0]; ry({t}) a[1]; rz({t}) b[0];
    u3({t},{p},{l}) a[0]; u2({p},{l}) a[1]; u1({l}) b[0];
    sdg a[0]; tdg a[1]; id b[0];
    cu1({l}) a[0],b[0]; cz a[1],b[0]; cp(pi/3) b[0],a[0];"""
    n, g = qasm.parse_qasm(prog)
    assert n == 3
    c, s = math.cos(t / 2), math.sin(t / 2)
    mats = [
        (0, np.array([[c, -1j * s], [-1j * s, c]])),
        (1, np.array([[c, -s], [s, c]])),
        (2, np.diag([cmath.exp(-0.5j * t), cmath.exp(0.5j * t)])),
        (0, np.array([[c, -cmath.exp(1j * l) * s], [cmath.exp(1j * p) * s, cmath.exp(1j * (p + l)) * c]])),
        (1, np.array([[1, -cmath.exp(1j * l)], [cmath.exp(1j * p), cmath.exp(1j * (p + l))]]) / math.sqrt(2)),
        (2, np.diag([1, cmath.exp(1j * l)])),
        (0, np.diag([1, -1j])),
        (1, np.diag([1, cmath.exp(-1j * math.pi / 4)])),
    ]
    want = [W.gate(W.OP_U, q, u=m) for q, m in mats]
    want += [W.gate(W.OP_CP, 0, 2, theta=l), W.gate(W.OP_CZ, 1, 2), W.gate(W.OP_CP, 2, 0, theta=math.pi / 3)]
    rng = np.random.default_rng(3)
    psi0 = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    a = sv.run_circuit(n, g, psi=psi0.copy())
    b = sv.run_circuit(n, W.concat(*want), psi=psi0.copy())
    assert np.max(np.abs(a - b)) < 1e-14


def test_swap_broadcast_and_expressions():
    prog = """OPENQASM 2.0;
    qreg q[3]; qreg r[3];
    h q;                      // broadcast over a register
    x r[1];
    swap q[0], r[1];
    cx q, r;                  // pairwise over equal registers
    rz(-pi/2 + 2*sin(pi/6)^2) q[2];
    barrier q, r;"""
    n, g = qasm.parse_qasm(prog)
    assert n == 6
    # swap is three CNOTs; compare with the permuted state
    psi = sv.run_circuit(n, g)
    hand = W.concat(*[W.gate(W.OP_H, q) for q in range(3)], W.gate(W.OP_X, 4),
                    W.gate(W.OP_CNOT, 0, 4), W.gate(W.OP_CNOT, 4, 0), W.gate(W.OP_CNOT, 0, 4),
                    *[W.gate(W.OP_CNOT, q, 3 + q) for q in range(3)],
                    W.gate(W.OP_U, 2, u=np.diag([cmath.exp(-0.5j * (-math.pi / 2 + 0.5)),
                                                 cmath.exp(0.5j * (-math.pi / 2 + 0.5))])))
    assert np.max(np.abs(psi - sv.run_circuit(n, hand))) < 1e-14


@pytest.mark.parametrize("prog, what", [
    ("OPENQASM 2.0; qreg q[2]; measure q[0] -> c[0];", "not supported"),
    ("OPENQASM 2.0; qreg q[2]; ccx q[0],q[1],q[0];", "unsupported statement"),
    ("OPENQASM 2.0; qreg q[2]; h q[2];", "out of range"),
    ("OPENQASM 2.0; qreg q[2]; rx(1,2) q[0];", "parameters"),
    ("OPENQASM 2.0; qreg q[2]; rx(__import__('os')) q[0];", "expression"),
    ("OPENQASM 2.0; qreg q[2]; cx q[1],q[1];", "twice"),
    ("OPENQASM 3.0; qubit[2] q;", "version"),
    ("OPENQASM 2.0; creg c[2];", "no qreg"),
    ("OPENQASM 2.0; qreg q[2]; gate g a { h a; }", "not supported"),
])
def test_rejects(prog, what):
    with pytest.raises(qasm.QasmError) as e:
        qasm.parse_qasm(prog)
    assert what in str(e.value)
