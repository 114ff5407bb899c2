"""Pins of the cut-search oracle (Alg. 2-3, Table I, Eq. (6)): closed-form
partitions of disconnected and unconstrained circuits, hand-worked merges
where Table I's contraction-edge penalty (4^(x - K_t) + 1 above K_t, x / K_t
below) and the largest contraction-edge count K_trial between the trial and a
neighbour decide the partition, the hard constraints and termination on
random circuits, agreement of its width count with the wire cutter's
subcircuits, exactness of the found cuts (reconstruction equals the uncut
statevector), and Eq. (6) at hand-computed values."""
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


# A chain of four two-qubit gates CZ(0,1), CZ(1,2), CZ(2,3), CZ(3,4): DAG
# vertices v0..v3, edges e0 = v0-v1 (qubit 1), e1 = v1-v2 (qubit 2), e2 =
# v2-v3 (qubit 3).  Worked by hand with K_t = 1, w_max = 4, s_max = 100:
#   every first trial has w = 3, s = 2, and K_trial = 2: the union of its cut
#   edges with those of a neighbour (e.g. {v0,v1}: {e1} | cuts({v2}) = {e1,e2};
#   {v1,v2}: {e0,e2}), so its cost is 3/4 + 2/100 + (4^(2-1) + 1) = 5.77.
#   With Q_max = 6 the tie goes to (v0, v1); then {v0,v1,v2} costs
#   4/4 + 3/100 + 1/1 = 2.03 (its only neighbour v3 shares e2 alone), while
#   the untouched pair (v2, v3) keeps its earlier 5.77 (Alg. 2 updates only
#   the edges on the new partition), so v2 joins; adding v3 would make w = 5.
#   With Q_max = 5.5 no trial is allowed and every gate stays alone.
# Plausible misreadings give other partitions: K_trial = |cuts(T)| alone
# makes (v0,v1) and (v2,v3) cost 1.77 each -> [0, 0, 1, 1] at Q_max = 6;
# a penalty of 4^(x - K_t) without the +1 (4.77) or 2^(x - K_t) + 1 (3.77)
# lets merges through at Q_max = 5.5.
CHAIN4 = [(0, 1), (1, 2), (2, 3), (3, 4)]


def test_contraction_edge_penalty_decides_the_merge():
    lab = cutfind.greedy_graph_growing(5, CHAIN4, w_max=4, s_max=100, k_t=1, q_max=6.0)
    assert [lab[g] for g in range(4)] == [0, 0, 0, 1]


def test_penalty_plus_one_keeps_every_gate_alone_below_its_cutoff():
    lab = cutfind.greedy_graph_growing(5, CHAIN4, w_max=4, s_max=100, k_t=1, q_max=5.5)
    assert [lab[g] for g in range(4)] == [0, 1, 2, 3]


def test_below_threshold_contraction_edges_cost_x_over_t():
    # K_t = 2: every first trial costs 3/4 + 2/100 + 2/2 = 1.77 (ties to
    # (v0, v1)); then {v0,v1,v2} costs 1 + 0.03 + 1/2 = 1.53 < 1.77, and v3
    # cannot join (w = 5 > 4)
    lab = cutfind.greedy_graph_growing(5, CHAIN4, w_max=4, s_max=100, k_t=2, q_max=1e4)
    assert [lab[g] for g in range(4)] == [0, 0, 0, 1]
    # the same chain with a binding gate count: s_max = 2 stops at pairs
    lab = cutfind.greedy_graph_growing(5, CHAIN4, w_max=10, s_max=2, k_t=2, q_max=1e4)
    assert [lab[g] for g in range(4)] == [0, 0, 1, 1]


def test_qpu_runtime_worked_values():
    # Eq. (6) with the paper's t_g = 1e-7 s and t_m = 1e-6 s, worked by hand:
    # one uncut 10-qubit, 20-layer circuit: 1024 * (2e-6 + 1e-6) = 3.072e-3 s;
    # u = 1, d = 1, w = 3, t = 5: 3 * 4 * 8 * 1.5e-6 = 1.44e-4 s;
    # (u, d) = (2, 0) and (0, 2) at w = 4, t = 10: (144 + 256) * 2e-6 = 8e-4 s
    assert math.isclose(cutfind.qpu_runtime([(0, 0, 10, 20)]), 3.072e-3, rel_tol=1e-12)
    assert math.isclose(cutfind.qpu_runtime([(1, 1, 3, 5)]), 1.44e-4, rel_tol=1e-12)
    assert math.isclose(cutfind.qpu_runtime([(2, 0, 4, 10), (0, 2, 4, 10)]), 8.0e-4, rel_tol=1e-12)
