"""The library's cut search (tqc_find_cuts, host code) against the oracle's
greedy graph growing (Alg. 2-3, Table I): the same partition, gate for gate,
on brickwork, QAOA and grid circuits, with hard limits binding, with the
contraction-edge penalty binding (small K_t) and with Q_max cutting the
growth short."""
import math

import numpy as np
import pytest

import paper_2502_03445_amd as tqc
from oracle import cutfind
from workloads import batch
from workloads.circuit import Circuit
from workloads.qaoa import random_regular_graph


def brickwork(n, depth, seed):
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for layer in range(depth):
        for q in range(n):
            c.add("rz", q, params=(rng.uniform(0, 2 * math.pi),))
        for q in range(layer % 2, n - 1, 2):
            c.add("cz", q, q + 1)
    return c


def qaoa_circuit(n, seed):
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(n, 3, rng)
    c = Circuit(n)
    for q in range(n):
        c.add("h", q)
    for a, b in edges:
        c.add("rzz", int(a), int(b), params=(0.7,))
    for q in range(n):
        c.add("rx", q, params=(0.3,))
    return c


def circuits():
    out = [("brick12", brickwork(12, 6, 1)), ("brick16", brickwork(16, 8, 2)), ("qaoa16", qaoa_circuit(16, 3)),
           ("qaoa24", qaoa_circuit(24, 4))]
    for i in (3, 7):
        n, m, layout, depth, circ, sub, home, target = batch.draw(i)
        out.append((f"batch{i}", circ))
    return out


@pytest.mark.parametrize("w_max,s_max,k_t,q_max", [(6, 1000, 10, 1e4), (8, 12, 10, 1e4), (5, 20, 3, 1e4),
                                                   (10, 1000, 2, 30.0), (4, 6, 10, 2.0)])
def test_library_partition_equals_oracle(w_max, s_max, k_t, q_max):
    for name, c in circuits():
        gates = [g.qubits for g in c.gates]
        ref = cutfind.greedy_graph_growing(c.n, gates, w_max, s_max, k_t, q_max)
        labels, parts = tqc.find_cuts(c.n, gates, w_max, s_max, k_t, q_max)
        got = {g: int(l) for g, l in enumerate(labels) if l >= 0}
        assert got == ref, name
        assert parts == len(set(ref.values()))
        assert all(labels[g] == -1 for g, qs in enumerate(gates) if len(qs) == 1)


@pytest.mark.parametrize("w_max,s_max,k_t,q_max,want", [(4, 100, 1, 6.0, [0, 0, 0, 1]), (4, 100, 1, 5.5, [0, 1, 2, 3]),
                                                        (4, 100, 2, 1e4, [0, 0, 0, 1]), (10, 2, 2, 1e4, [0, 0, 1, 1])])
def test_library_on_hand_worked_chain(w_max, s_max, k_t, q_max, want):
    # the chain CZ(0,1), CZ(1,2), CZ(2,3), CZ(3,4) worked by hand from
    # Table I (tests/test_oracle_cutfind.py explains each partition)
    labels, parts = tqc.find_cuts(5, [(0, 1), (1, 2), (2, 3), (3, 4)], w_max, s_max, k_t, q_max)
    assert list(labels) == want and parts == len(set(want))


def test_find_cuts_rejects_bad_input():
    with pytest.raises(tqc.TqcError):
        tqc.find_cuts(4, [(0, 5)], 4, 10)
    with pytest.raises(tqc.TqcError):
        tqc.find_cuts(4, [(1, 1)], 4, 10)
    with pytest.raises(tqc.TqcError):
        tqc.find_cuts(4, [(0, 1)], 0, 10)
