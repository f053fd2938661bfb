"""Circuit front-end: an OpenQASM 2.0 subset to gate records (the
``juqcs_gate`` layout of include/juqcs_gpu.h, ``workloads.GATE_DTYPE``).

The paper's simulator reads circuits in its own instruction set (Section 2);
this front-end takes the common interchange text instead and produces the
same gate records that the rest of the package consumes.

Supported: the ``OPENQASM 2.0;`` header, ``include "qelib1.inc";``, ``qreg``
(several registers are numbered one after the other), ``creg`` and
``barrier`` (ignored), and the gates

    id x y z h s sdg t tdg rx ry rz u1 u2 u3 u U p
    cx CX cz cp cu1 swap

with parameter expressions over numbers, ``pi``, + - * / ^ (and **), unary
minus and sin cos tan exp ln sqrt.  A gate applied to whole registers is
broadcast (one-qubit gates over a register, two-qubit gates pairwise over
registers of equal size).  ``measure``, ``reset``, ``if``, ``opaque`` and
``gate`` definitions raise QasmError: the simulator returns amplitudes, not
measurement records.

Conventions (qelib1): u3(t, p, l) = [[cos t/2, -e^{il} sin t/2],
[e^{ip} sin t/2, e^{i(p+l)} cos t/2]]; u2(p, l) = u3(pi/2, p, l);
u1(l) = p(l) = diag(1, e^{il}); rx, ry, rz are exp(-i t sigma/2);
cu1(l) = cp(l) = diag(1, 1, 1, e^{il}); swap a, b = cx a,b; cx b,a; cx a,b.
"""
import ast
import math
import re

import numpy as np

from . import workloads as W


class QasmError(ValueError):
    pass


_FUNCS = {"sin": math.sin, "cos": math.cos, "tan": math.tan, "exp": math.exp, "ln": math.log,
          "sqrt": math.sqrt}


def _eval(expr: str) -> float:
    """Value of a parameter expression (an AST walk: nothing is executed)."""
    try:
        tree = ast.parse(expr.replace("^", "**"), mode="eval")
    except SyntaxError as e:
        raise QasmError(f"bad expression {expr!r}") from e

    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return float(node.value)
        if isinstance(node, ast.Name) and node.id == "pi":
            return math.pi
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
            v = ev(node.operand)
            return -v if isinstance(node.op, ast.USub) else v
        if isinstance(node, ast.BinOp):
            a, b = ev(node.left), ev(node.right)
            if isinstance(node.op, ast.Add):
                return a + b
            if isinstance(node.op, ast.Sub):
                return a - b
            if isinstance(node.op, ast.Mult):
                return a * b
            if isinstance(node.op, ast.Div):
                return a / b
            if isinstance(node.op, ast.Pow):
                return a ** b
        if (isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id in _FUNCS
                and len(node.args) == 1 and not node.keywords):
            return _FUNCS[node.func.id](ev(node.args[0]))
        raise QasmError(f"unsupported expression {expr!r}")

    return ev(tree)


def _u3(t: float, p: float, l: float) -> np.ndarray:
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -np.exp(1j * l) * s], [np.exp(1j * p) * s, np.exp(1j * (p + l)) * c]])


def _one_qubit(name: str, args):
    """(op, matrix or None) of a one-qubit gate."""
    fixed = {"x": W.OP_X, "y": W.OP_Y, "z": W.OP_Z, "h": W.OP_H, "s": W.OP_S, "t": W.OP_T}
    if name in fixed:
        return fixed[name], None
    if name == "id":
        return None, None
    if name == "sdg":
        return W.OP_U, np.diag([1.0, -1j])
    if name == "tdg":
        return W.OP_U, np.diag([1.0, np.exp(-1j * math.pi / 4)])
    if name in ("u3", "u", "U"):
        return W.OP_U, _u3(*args)
    if name == "u2":
        return W.OP_U, _u3(math.pi / 2, *args)
    if name in ("u1", "p"):
        return W.OP_U, np.diag([1.0, np.exp(1j * args[0])])
    if name == "rx":
        c, s = math.cos(args[0] / 2), math.sin(args[0] / 2)
        return W.OP_U, np.array([[c, -1j * s], [-1j * s, c]])
    if name == "ry":
        c, s = math.cos(args[0] / 2), math.sin(args[0] / 2)
        return W.OP_U, np.array([[c, -s], [s, c]])
    if name == "rz":
        return W.OP_U, np.diag([np.exp(-0.5j * args[0]), np.exp(0.5j * args[0])])
    raise KeyError(name)


_NPARAMS = {"id": 0, "x": 0, "y": 0, "z": 0, "h": 0, "s": 0, "sdg": 0, "t": 0, "tdg": 0, "rx": 1,
            "ry": 1, "rz": 1, "u1": 1, "p": 1, "u2": 2, "u3": 3, "u": 3, "U": 3, "cx": 0, "CX": 0,
            "cz": 0, "cp": 1, "cu1": 1, "swap": 0}
_TWO = ("cx", "CX", "cz", "cp", "cu1", "swap")


def _split_args(text: str):
    """Top-level comma split (commas inside parentheses stay)."""
    out, depth, cur = [], 0, ""
    for ch in text:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == "," and depth == 0:
            out.append(cur)
            cur = ""
        else:
            cur += ch
    if cur.strip():
        out.append(cur)
    return [a.strip() for a in out]


def parse_qasm(text: str):
    """(n, gate records) of an OpenQASM 2.0 program (subset in the module
    docstring).  Raises QasmError on anything outside the subset."""
    text = re.sub(r"//[^\n]*", "", text)
    stmts = [s.strip() for s in text.split(";")]
    regs = {}  # name -> (offset, size)
    n = 0
    recs = []

    def qubits(ref: str):
        m = re.fullmatch(r"([A-Za-z_]\w*)\s*(\[\s*(\d+)\s*\])?", ref)
        if not m or m.group(1) not in regs:
            raise QasmError(f"unknown qubit reference {ref!r}")
        off, size = regs[m.group(1)]
        if m.group(2) is None:
            return [off + i for i in range(size)]
        i = int(m.group(3))
        if i >= size:
            raise QasmError(f"index {i} out of range for register {m.group(1)}[{size}]")
        return [off + i]

    for st in stmts:
        if not st:
            continue
        head = st.split(None, 1)[0]
        if head == "OPENQASM":
            if not re.fullmatch(r"OPENQASM\s+2(\.0)?", st):
                raise QasmError(f"unsupported version: {st!r}")
            continue
        if head == "include":
            continue
        if head in ("qreg", "creg"):
            m = re.fullmatch(r"(qreg|creg)\s+([A-Za-z_]\w*)\s*\[\s*(\d+)\s*\]", st)
            if not m:
                raise QasmError(f"bad register declaration {st!r}")
            if head == "qreg":
                if m.group(2) in regs:
                    raise QasmError(f"register {m.group(2)} declared twice")
                regs[m.group(2)] = (n, int(m.group(3)))
                n += int(m.group(3))
            continue
        if head == "barrier":
            continue
        if head in ("measure", "reset", "if", "opaque", "gate") or head.startswith("if("):
            raise QasmError(f"{head!r} is not supported (the simulator returns amplitudes)")
        m = re.fullmatch(r"([A-Za-z_]\w*)\s*(\((.*)\))?\s*(.*)", st, flags=re.S)
        if not m or m.group(1) not in _NPARAMS:
            raise QasmError(f"unsupported statement {st!r}")
        name = m.group(1)
        params = [_eval(a) for a in _split_args(m.group(3))] if m.group(2) else []
        if len(params) != _NPARAMS[name]:
            raise QasmError(f"{name} takes {_NPARAMS[name]} parameters, got {len(params)}")
        targets = [qubits(a) for a in _split_args(m.group(4))]
        if name in _TWO:
            if len(targets) != 2:
                raise QasmError(f"{name} acts on two qubits: {st!r}")
            a, b = targets
            if len(a) != len(b) and min(len(a), len(b)) != 1:
                raise QasmError(f"register sizes differ in {st!r}")
            k = max(len(a), len(b))
            for i in range(k):
                qa, qb = a[i if len(a) > 1 else 0], b[i if len(b) > 1 else 0]
                if qa == qb:
                    raise QasmError(f"{name} on one qubit twice: {st!r}")
                if name in ("cx", "CX"):
                    recs.append(W.gate(W.OP_CNOT, qa, qb))
                elif name == "cz":
                    recs.append(W.gate(W.OP_CZ, qa, qb))
                elif name in ("cp", "cu1"):
                    recs.append(W.gate(W.OP_CP, qa, qb, theta=params[0]))
                else:  # swap
                    recs += [W.gate(W.OP_CNOT, qa, qb), W.gate(W.OP_CNOT, qb, qa),
                             W.gate(W.OP_CNOT, qa, qb)]
        else:
            if len(targets) != 1:
                raise QasmError(f"{name} acts on one qubit: {st!r}")
            op, u = _one_qubit(name, params)
            for q in targets[0]:
                if op is not None:
                    recs.append(W.gate(op, q, u=u))
    if n == 0:
        raise QasmError("no qreg declared")
    return n, W.concat(*recs)
