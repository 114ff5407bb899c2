"""Gate-list circuits and a dense complex128 statevector simulator.

This module stands in for the quantum processors of the method (Sec. II-A):
it produces the measured probability vectors of circuits and subcircuits.
It holds none of the reconstruction arithmetic (no Pauli-basis transform and
no contraction), so both the oracle and the GPU path may take its outputs as
inputs.

Bit convention: in a statevector over w qubits, qubit q is bit q of the
basis-state index (qubit 0 is the least significant bit).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_SQ2 = 1.0 / np.sqrt(2.0)


def _rx(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def _ry(t):
    c, s = np.cos(t / 2), np.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def _rz(t):
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


ONE_QUBIT = {
    "h": lambda: np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128),
    "x": lambda: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "y": lambda: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "z": lambda: np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "s": lambda: np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "sdg": lambda: np.array([[1, 0], [0, -1j]], dtype=np.complex128),
    "t": lambda: np.array([[1, 0], [0, np.exp(0.25j * np.pi)]], dtype=np.complex128),
    # square roots of X and Y (the random-circuit gate set of Google-style circuits)
    "sx": lambda: 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128),
    "sy": lambda: 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128),
    "rx": _rx,
    "ry": _ry,
    "rz": _rz,
}


def _two_qubit(name, params):
    """4x4 unitary on (q_a, q_b) in the basis index = b_a + 2*b_b."""
    if name == "cz":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "cx":  # control = first qubit, target = second
        u = np.zeros((4, 4), dtype=np.complex128)
        for ba in range(2):
            for bb in range(2):
                u[ba + 2 * (bb ^ ba), ba + 2 * bb] = 1
        return u
    if name == "rzz":  # exp(-i theta/2 Z(x)Z)
        t = params[0]
        ph = [np.exp(-0.5j * t * (1 - 2 * (ba ^ bb))) for bb in range(2) for ba in range(2)]
        return np.diag(ph).astype(np.complex128)
    if name == "cp":  # controlled phase
        return np.diag([1, 1, 1, np.exp(1j * params[0])]).astype(np.complex128)
    if name == "cry":  # controlled Ry: control = first qubit, target = second
        r = _ry(params[0])
        u = np.eye(4, dtype=np.complex128)
        # states with control bit (ba) = 1: indices 1 (bb=0) and 3 (bb=1)
        u[np.ix_([1, 3], [1, 3])] = r
        return u
    raise ValueError(f"unknown two-qubit gate {name}")


@dataclass
class Gate:
    name: str
    qubits: tuple
    params: tuple = ()

    def matrix(self):
        if len(self.qubits) == 1:
            f = ONE_QUBIT[self.name]
            return f(*self.params) if self.params else f()
        return _two_qubit(self.name, self.params)


@dataclass
class Circuit:
    n: int
    gates: list = field(default_factory=list)

    def add(self, name, *qubits, params=()):
        self.gates.append(Gate(name, tuple(qubits), tuple(params)))
        return self


def apply_1q(psi, w, q, u):
    v = psi.reshape(1 << (w - q - 1), 2, 1 << q)
    return np.einsum("ab,xby->xay", u, v).reshape(-1)


def apply_2q(psi, w, qa, qb, u):
    """u acts on (qa, qb) with local index b_qa + 2*b_qb."""
    t = psi.reshape([2] * w)  # axis k <-> qubit w-1-k
    ax_a, ax_b = w - 1 - qa, w - 1 - qb
    t = np.moveaxis(t, (ax_b, ax_a), (0, 1))  # shape (2_b, 2_a, ...)
    sh = t.shape
    m = t.reshape(4, -1)  # row index = 2*b_b + b_a
    m = u @ m
    t = m.reshape(sh)
    t = np.moveaxis(t, (0, 1), (ax_b, ax_a))
    return np.ascontiguousarray(t).reshape(-1)


def apply_gate(psi, w, gate, qmap=None):
    qs = gate.qubits if qmap is None else tuple(qmap[q] for q in gate.qubits)
    u = gate.matrix()
    if len(qs) == 1:
        return apply_1q(psi, w, qs[0], u)
    return apply_2q(psi, w, qs[0], qs[1], u)


def statevector(circ: Circuit, psi0=None):
    w = circ.n
    if psi0 is None:
        psi = np.zeros(1 << w, dtype=np.complex128)
        psi[0] = 1.0
    else:
        psi = np.array(psi0, dtype=np.complex128)
    for g in circ.gates:
        psi = apply_gate(psi, w, g)
    return psi


def probabilities(circ: Circuit):
    psi = statevector(circ)
    return (psi.real ** 2 + psi.imag ** 2)
