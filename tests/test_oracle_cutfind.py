"""Pins of the cut-search oracle (Alg. 2-3, Table I, Eq. (6)): closed-form
partitions of disconnected and unconstrained circuits, the hard constraints
and termination on random circuits, agreement of its width count with the
wire cutter's subcircuits, and exactness of the found cuts (reconstruction
equals the uncut statevector)."""
import math

import numpy as np

from oracle import cutfind
from oracle.reconstruct import full_distribution
from workloads.circuit import Circuit, probabilities
from workloads.cutting import assign_from_partition, cut_circuit, cut_shapes


def brickwork(n, depth, seed, blocks=None):
    """Rx/Ry/Rz layers and nearest-neighbour CZ brickwork; `blocks` (list of
    qubit ranges) keeps the CZs inside each block."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    block_of = {}
    for b, (lo, hi) in enumerate(blocks or [(0, n)]):
        for q in range(lo, hi):
            block_of[q] = b
    for layer in range(depth):
        for q in range(n):
            c.add(("rx", "ry", "rz")[rng.integers(3)], q, params=(rng.uniform(0, 2 * math.pi),))
        for q in range(layer % 2, n - 1, 2):
            if block_of[q] == block_of[q + 1]:
                c.add("cz", q, q + 1)
    return c


def gates_of(c):
    return [g.qubits for g in c.gates]


def test_disconnected_blocks_become_two_uncut_partitions():
    c = brickwork(8, 5, 1, blocks=[(0, 4), (4, 8)])
    lab = cutfind.greedy_graph_growing(8, gates_of(c), w_max=4, s_max=1000)
    parts = {}
    for g, p in lab.items():
        parts.setdefault(p, set()).update(c.gates[g].qubits)
    assert sorted(map(sorted, parts.values())) == [[0, 1, 2, 3], [4, 5, 6, 7]]
    gs, idle, m = assign_from_partition(c, lab)
    cuts, _ = cut_shapes(c, gs, num_subs=m, idle_sub=idle)
    assert cuts == []


def test_unconstrained_line_merges_into_one_partition():
    c = brickwork(6, 4, 2)
    lab = cutfind.greedy_graph_growing(6, gates_of(c), w_max=6, s_max=1000)
    assert set(lab.values()) == {0}


def test_constraints_termination_and_exact_cuts():
    exact = 0
    for seed, (n, depth, w_max, s_max) in enumerate([(8, 5, 5, 40), (9, 5, 4, 12), (10, 5, 6, 9), (8, 5, 3, 100),
                                                     (6, 3, 4, 100), (8, 3, 6, 100), (7, 2, 4, 100)]):
        c = brickwork(n, depth, 10 + seed)
        g = gates_of(c)
        lab = cutfind.greedy_graph_growing(n, g, w_max=w_max, s_max=s_max)
        verts, edges = cutfind.dag_of(n, g)
        vid = {gg: v for v, gg in enumerate(verts)}
        parts = {}
        for gg, p in lab.items():
            parts.setdefault(p, set()).add(vid[gg])
        gs, idle, m = assign_from_partition(c, lab)
        cuts, shapes = cut_shapes(c, gs, num_subs=m, idle_sub=idle)
        for p, members in parts.items():
            w = cutfind._width(members, verts, g)
            assert w <= w_max and len(members) <= s_max
            # the width count is the wire cutter's subcircuit width
            assert w == shapes[p]["width"] - sum(1 for q in range(n) if idle[q] == p and
                                                 all(len(gt.qubits) == 1 or q not in gt.qubits
                                                     for gt in c.gates)), (p, w, shapes[p])
        # no adjacent pair could still merge within the hard limits (these
        # circuits never reach K_t = 10 contraction edges, so only w_max and
        # s_max can stop the growth)
        for a, b, _ in edges:
            pa = [p for p, ms in parts.items() if a in ms][0]
            pb = [p for p, ms in parts.items() if b in ms][0]
            if pa == pb:
                continue
            union = parts[pa] | parts[pb]
            assert (cutfind._width(union, verts, g) > w_max or len(union) > s_max)
        # the cuts are exact: reconstruction equals the uncut statevector
        if max(s["width"] for s in shapes) <= 10 and len(cuts) <= 6:
            net = cut_circuit(c, gs, num_subs=m, idle_sub=idle)
            assert np.abs(full_distribution(net) - probabilities(c)).max() <= 1e-12
            exact += 1
    assert exact >= 3


def test_qpu_runtime_of_one_uncut_circuit():
    # Eq. (6) with no cuts: 2^w shots of (t layers * t_g + t_m)
    assert math.isclose(cutfind.qpu_runtime([(0, 0, 10, 20)]), 2 ** 10 * (20e-7 + 1e-6))
    assert math.isclose(cutfind.qpu_runtime([(1, 2, 3, 4)]), 3 * 16 * 8 * (4e-7 + 1e-6))
