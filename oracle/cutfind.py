"""Greedy Graph Growing cut search (Sec. VI, Alg. 2-3, Table I) and the
runtime estimates of Eqs. (6)-(8).

TEST INFRASTRUCTURE ONLY (see the package header).

Readings (the paper leaves these open):
* DAG: one vertex per two-qubit gate (circuit order = vertex id); one edge
  per wire segment between consecutive two-qubit gates of a qubit (edge id
  in order of (earlier gate, later gate, qubit)).  Single-qubit gates and
  the input / output vertices ride with their neighbouring two-qubit gates.
* Partition metrics: s = its two-qubit gates; w = its qubits, one per
  maximal run of a wire's two-qubit gates inside it (a wire that leaves and
  comes back is a second qubit, as wire cutting makes it); cuts(P) = DAG
  edges with exactly one end in P; the contraction edges of neighbours P, Q
  are cuts(P) | cuts(Q) (internal and external, Sec. III-C).
* Merging cost of a pair (Alg. 3, Table I): for the trial union T,
  c(w_T; w_max) + c(s_T; s_max) + c(K_T; K_t) with K_T = the largest
  contraction-edge count between T and one of its neighbours (0 without
  neighbours); c = x / T at or below the threshold, not allowed above it
  for w and s, 4^(x - T) + 1 above it for K.
* Alg. 2: every adjacent pair of partitions is costed once (all its edges
  give the same trial); the cheapest pair with cost <= Q_max is merged
  (ties: smaller (first vertex of one side, first vertex of the other));
  after a merge only the pairs touching the merged partition are costed
  again, the others keep their earlier cost, as the algorithm states; it
  stops when no pair is allowed.
* Eq. (6): T_QPU = sum_i 3^u_i 4^d_i 2^w_i (t_i t_g + t_m) with t_g = 1e-7 s,
  t_m = 1e-6 s, t_i = gate layers of subcircuit i; Eq. (7): T_classical =
  contraction flops / device flop rate; Eq. (8): T = T_QPU + T_classical.
"""
from __future__ import annotations

import math


def dag_of(num_qubits, gates):
    """gates: list of qubit tuples in circuit order.  Returns (vertex gate
    indices, edges [(a, b, qubit)] between vertex ids)."""
    verts = [g for g, qs in enumerate(gates) if len(qs) == 2]
    vid = {g: v for v, g in enumerate(verts)}
    last = [-1] * num_qubits
    edges = []
    for g in verts:
        for q in gates[g]:
            if last[q] >= 0:
                edges.append((vid[last[q]], vid[g], q))
            last[q] = g
    edges.sort()
    return verts, edges


def _width(part, verts, gates):
    """qubits of a set of vertices: maximal runs of each wire's 2q gates"""
    wires = {}
    for v, g in enumerate(verts):
        for q in gates[g]:
            wires.setdefault(q, []).append(v)
    runs = 0
    for q, vs in wires.items():
        inside = False
        for v in vs:
            if v in part and not inside:
                runs += 1
            inside = v in part
    return runs


def _cost(x, thr, hard):
    if x <= thr:
        return x / thr
    if hard or x - thr >= 512:  # 4^512 overflows a double
        return math.inf
    return 4.0 ** (x - thr) + 1.0


def greedy_graph_growing(num_qubits, gates, w_max, s_max, k_t=10, q_max=1e4):
    """Partition label of every two-qubit gate (by circuit gate index), labels
    0.. in order of each partition's first gate."""
    verts, edges = dag_of(num_qubits, gates)
    label = list(range(len(verts)))          # partition id of each vertex
    members = {v: {v} for v in range(len(verts))}

    def cuts_of(p):
        return {e for e, (a, b, _) in enumerate(edges) if (label[a] == p) != (label[b] == p)}

    def neighbours(pset):
        out = set()
        for a, b, _ in edges:
            la, lb = label[a], label[b]
            if (a in pset) != (b in pset):
                out.add(lb if a in pset else la)
        return out

    def trial_cost(p, q):
        t = members[p] | members[q]
        w = _width(t, verts, gates)
        s = len(t)
        tc = {e for e, (a, b, _) in enumerate(edges) if (a in t) != (b in t)}
        k = 0
        for r in neighbours(t):
            k = max(k, len(tc | cuts_of(r)))
        return _cost(w, w_max, True) + _cost(s, s_max, True) + _cost(k, k_t, False)

    def pairs():
        ps = set()
        for a, b, _ in edges:
            la, lb = label[a], label[b]
            if la != lb:
                ps.add((min(la, lb), max(la, lb)))
        return ps

    cost = {pq: trial_cost(*pq) for pq in pairs()}
    while True:
        live = pairs()
        best = None
        for pq in live:
            c = cost[pq]
            if c > q_max:
                continue
            key = (c,) + tuple(sorted((min(members[pq[0]]), min(members[pq[1]]))))
            if best is None or key < best[0]:
                best = (key, pq)
        if best is None:
            break
        p, q = best[1]
        members[p] |= members.pop(q)
        for v in members[p]:
            label[v] = p
        # the merged partition keeps id p; pairs touching it are costed again
        for pq in list(cost):
            if q in pq or pq not in pairs():
                cost.pop(pq, None)
        for pq in pairs():
            if p in pq or pq not in cost:
                cost[pq] = trial_cost(*pq)
    # labels in order of first gate
    order = sorted(members, key=lambda p: min(members[p]))
    ren = {p: i for i, p in enumerate(order)}
    return {verts[v]: ren[label[v]] for v in range(len(verts))}


def qpu_runtime(subcircuits, t_g=1e-7, t_m=1e-6):
    """Eq. (6): subcircuits = [(u, d, w, layers)]."""
    return sum(3 ** u * 4 ** d * 2 ** w * (t * t_g + t_m) for u, d, w, t in subcircuits)
