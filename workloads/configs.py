"""Seeded workload builders.

Base seed 20250205 plus the workload number; numpy SeedSequence streams.
Circuits are built from their textbook descriptions (Sec. VII-B families:
QAOA on random 3-regular graphs, AQFT, GHZ, W state, random circuits) and
cut constructively by assigning gates to subcircuits.
"""
from __future__ import annotations

import numpy as np

from .circuit import Circuit
from .cutting import cut_circuit

BASE_SEED = 20250205


def rng_for(config: int, stream: int = 0, seed=None):
    # the stream-th child of SeedSequence(base) (what .spawn() would hand out)
    entropy = BASE_SEED + config if seed is None else seed
    return np.random.default_rng(np.random.SeedSequence(entropy, spawn_key=(stream,)))


# ---------------------------------------------------------------- tiny line

def line_circuit_12(seed=None):
    """12-qubit line, 4 layers of Rx.Ry.Rz with U[0,2pi) angles then CZ on
    nearest-neighbour bonds; bond (5,6) carries its CZ in layer 1 only, so the
    middle wire can be cut just before and just after that one gate."""
    rng = rng_for(1, 0, seed)
    n = 12
    c = Circuit(n)
    for layer in range(4):
        for q in range(n):
            a, b, g = rng.uniform(0, 2 * np.pi, size=3)
            for name, ang in (("rx", a), ("ry", b), ("rz", g)):
                c.add(name, q, params=(ang,))
        for q in range(n - 1):
            if q == 5 and layer != 0:
                continue
            c.add("cz", q, q + 1)
    # subcircuit A (0): qubits 0..5 and the single CZ(5,6); B (1): the rest,
    # including every other gate on qubit 6
    sub = []
    for g in c.gates:
        qs = g.qubits
        if qs == (5, 6) or max(qs) <= 5:
            sub.append(0)
        else:
            sub.append(1)
    return c, sub


def config1(seed=None):
    c, sub = line_circuit_12(seed)
    net = cut_circuit(c, sub, num_subs=2)
    net.meta["circuit"] = c
    net.meta["name"] = "line12_4layer_2cut"
    return net


# ------------------------------------------------------- closed-form circuits

def _contiguous_groups(n, m):
    s = -(-n // m)
    return [min(q // s, m - 1) for q in range(n)]


def ghz(n, m):
    """GHZ chain H(0), CX(i,i+1); CX across a group boundary belongs to the
    group of its target, so the control wire migrates (one cut per boundary).
    Closed form: P(0..0) = P(1..1) = 1/2."""
    home = _contiguous_groups(n, m)
    c = Circuit(n)
    sub = []
    c.add("h", 0)
    sub.append(home[0])
    for i in range(n - 1):
        c.add("cx", i, i + 1)
        sub.append(home[i + 1])
    net = cut_circuit(c, sub, num_subs=m, idle_sub=home)
    net.meta.update(circuit=c, name=f"ghz{n}_{m}")
    return net


def w_state(n, m):
    """Linear W-state preparation: X(0); for each i a controlled Ry from q_i to
    q_{i+1} with cos(theta/2) = sqrt(1/(n-i)), then CX(q_{i+1}, q_i).
    Closed form: P(e_i) = 1/n for each one-hot e_i."""
    home = _contiguous_groups(n, m)
    c = Circuit(n)
    sub = []
    c.add("x", 0)
    sub.append(home[0])
    for i in range(n - 1):
        th = 2 * np.arccos(np.sqrt(1.0 / (n - i)))
        c.add("cry", i, i + 1, params=(th,))
        sub.append(home[i + 1])
        c.add("cx", i + 1, i)
        sub.append(home[i + 1])
    net = cut_circuit(c, sub, num_subs=m, idle_sub=home)
    net.meta.update(circuit=c, name=f"w{n}_{m}")
    return net


def aqft(n, m, degree=2, seed=None):
    """Approximate QFT (controlled phases between qubits at most `degree`
    apart) on a seeded basis state.  A QFT-type circuit on a basis state gives
    a product of equal-weight single-qubit superpositions, so P(x) = 2^-n for
    every x.  A controlled phase across a group boundary belongs to the group
    of its control, so the target wire migrates after its Hadamard."""
    rng = rng_for(90, 0, seed)
    home = _contiguous_groups(n, m)
    c = Circuit(n)
    sub = []
    for q in np.nonzero(rng.integers(0, 2, size=n))[0]:
        c.add("x", int(q))
        sub.append(home[int(q)])
    for j in range(n):
        c.add("h", j)
        sub.append(home[j])
        for k in range(j + 1, min(n, j + degree + 1)):
            c.add("cp", k, j, params=(np.pi / 2 ** (k - j),))
            sub.append(home[k])
    net = cut_circuit(c, sub, num_subs=m, idle_sub=home)
    net.meta.update(circuit=c, name=f"aqft{n}_{m}_d{degree}")
    return net


# -------------------------------------------------------- random small circuits

def random_cut_circuit(n, m, layers, max_cross, seed):
    """Random Rx/Ry/Rz + CZ/CX/RZZ circuit on n qubits split into m groups.
    Each two-qubit gate goes to the group of one of its qubits (seeded); a
    single-qubit gate goes to the wire's home group.  At most `max_cross`
    gates span groups, so the number of cuts stays small."""
    rng = np.random.default_rng(seed)
    home = [int(q * m // n) for q in range(n)]
    c = Circuit(n)
    sub = []
    cross = 0
    for _ in range(layers):
        for q in range(n):
            name = ("rx", "ry", "rz")[rng.integers(3)]
            c.add(name, q, params=(rng.uniform(0, 2 * np.pi),))
            sub.append(home[q])
        perm = rng.permutation(n)
        for a, b in zip(perm[0::2], perm[1::2]):
            a, b = int(a), int(b)
            if home[a] != home[b]:
                if cross >= max_cross:
                    continue
                cross += 1
            name = ("cz", "cx", "rzz")[rng.integers(3)]
            params = (rng.uniform(0, 2 * np.pi),) if name == "rzz" else ()
            c.add(name, a, b, params=params)
            sub.append(home[a] if rng.integers(2) else home[b])
    net = cut_circuit(c, sub, num_subs=m, idle_sub=home)
    net.meta.update(circuit=c, name=f"rand{n}_{m}_{seed}")
    return net
