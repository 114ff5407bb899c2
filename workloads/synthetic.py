"""Synthetic Pauli-basis tensor networks (the paper substitutes random numbers
for subcircuit outputs of large benchmarks, Sec. VII-A).

Values per tensor j: the all-I row T_j[I..I, :] ~ Dirichlet(alpha * 1) over
its 2^{o_j} columns; every other row T_j[sigma, x] ~ U[-p(x), p(x)] with p the
all-I row.  These are not physical distributions: the reconstructed vector
can be negative and need not sum to 1.
"""
from __future__ import annotations

import numpy as np

from .cutting import Network, TensorSpec


def regular_multigraph(num_nodes, degree, rng, max_tries=10000):
    """Configuration model without self-loops (multi-edges allowed)."""
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(num_nodes), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.all(pairs[:, 0] != pairs[:, 1]):
            return [(int(a), int(b)) for a, b in pairs]
    raise RuntimeError("no loop-free multigraph")


def tensor_values(num_cuts, num_outputs, rng, alpha=0.1):
    cols = 1 << num_outputs
    T = np.empty((4 ** num_cuts, cols), dtype=np.float64)
    p = rng.dirichlet(np.full(cols, alpha))
    T[0] = p
    if num_cuts:
        T[1:] = rng.uniform(-1.0, 1.0, size=(4 ** num_cuts - 1, cols)) * p
    return T


def network_from_edges(n, num_tensors, edges, outputs_per_tensor, rng, alpha=0.1):
    """edges: list of (a, b) tensor pairs, one per cut; orientation seeded."""
    cuts = []
    for a, b in edges:
        cuts.append((a, b) if rng.integers(2) else (b, a))
    qubits = rng.permutation(n)
    tensors = []
    pos = 0
    for j in range(num_tensors):
        o = outputs_per_tensor[j]
        outs = sorted(int(q) for q in qubits[pos:pos + o])
        pos += o
        cids = [c for c, (u, d) in enumerate(cuts) if j in (u, d)]
        T = tensor_values(len(cids), o, rng, alpha)
        tensors.append(TensorSpec(cut_ids=cids, outputs=outs, basis="pauli", data=T))
    assert pos == n
    return Network(n=n, cuts=cuts, tensors=tensors)


def precision_network(seed=None):
    """6 tensors, 18 cuts (a 6-regular multigraph: every tensor has exactly 6
    cuts), 34 output qubits split [6,6,6,6,5,5] in seeded order, 4 qubits fixed
    to seeded values (a 2^30 slice)."""
    from .configs import rng_for
    rng = rng_for(3, 0, seed)
    edges = regular_multigraph(6, 6, rng)
    net = network_from_edges(34, 6, edges, [6, 6, 6, 6, 5, 5], rng)
    fq = sorted(int(q) for q in rng.choice(34, size=4, replace=False))
    fv = [int(v) for v in rng.integers(0, 2, size=4)]
    net.meta.update(name="synthetic6_18cut_34q", fixed_qubits=fq, fixed_values=fv)
    return net


def random_network(num_tensors, num_cuts, outputs_per_tensor, seed, alpha=0.1,
                   connected=True):
    """Random connected multigraph network (spanning tree first, then extra
    edges) for tests."""
    rng = np.random.default_rng(seed)
    edges = []
    if connected:
        for j in range(1, num_tensors):
            edges.append((int(rng.integers(j)), j))
    while len(edges) < num_cuts:
        a, b = rng.choice(num_tensors, size=2, replace=False)
        edges.append((int(a), int(b)))
    n = int(sum(outputs_per_tensor))
    return network_from_edges(n, num_tensors, edges[:num_cuts], outputs_per_tensor, rng, alpha)


def grid_patch_network(seed=None, rows=2, cols=6, patch_h=5, patch_w=2, num_cuts=40,
                       free_per_patch=2):
    """Cut network of a 10x12 grid circuit split into a 2x6 arrangement of
    5x2-qubit patches (120 qubits, 12 subcircuits).  Cut edges join adjacent
    patches only; multiplicities are seeded so that corner patches carry 6 cuts
    and the other patches 7 (40 cuts, 80 endpoints).  Tensors are synthetic
    (Dirichlet(0.1) all-I row, uniform [-p, p] elsewhere); 2 seeded qubits per
    patch stay free and the other 96 are fixed to a seeded bitstring."""
    from .configs import rng_for
    rng = rng_for(5, 0, seed)
    P = rows * cols
    pid = lambda r, c: r * cols + c
    pairs = []
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                pairs.append((pid(r, c), pid(r, c + 1)))
            if r + 1 < rows:
                pairs.append((pid(r, c), pid(r + 1, c)))
    corners = {pid(0, 0), pid(0, cols - 1), pid(rows - 1, 0), pid(rows - 1, cols - 1)}
    target = [6 if j in corners else 7 for j in range(P)]
    assert sum(target) == 2 * num_cuts
    for _ in range(10000):
        mult = {e: 1 for e in pairs}
        deg = [0] * P
        for a, b in pairs:
            deg[a] += 1
            deg[b] += 1
        ok = True
        while sum(deg) < 2 * num_cuts:
            cand = [e for e in pairs if deg[e[0]] < target[e[0]] and deg[e[1]] < target[e[1]]]
            if not cand:
                ok = False
                break
            a, b = cand[int(rng.integers(len(cand)))]
            mult[(a, b)] += 1
            deg[a] += 1
            deg[b] += 1
        if ok and deg == target:
            break
    else:
        raise RuntimeError("no multiplicity assignment")
    edges = []
    for e in pairs:
        edges += [e] * mult[e]
    order = rng.permutation(len(edges))
    edges = [edges[i] for i in order]
    cuts = [(a, b) if rng.integers(2) else (b, a) for a, b in edges]
    n = rows * patch_h * cols * patch_w
    width = cols * patch_w
    tensors = []
    free = []
    for r in range(rows):
        for c in range(cols):
            j = pid(r, c)
            qs = sorted((r * patch_h + i) * width + (c * patch_w + k)
                        for i in range(patch_h) for k in range(patch_w))
            cids = [ci for ci, (u, d) in enumerate(cuts) if j in (u, d)]
            T = tensor_values(len(cids), len(qs), rng)
            tensors.append(TensorSpec(cut_ids=cids, outputs=qs, basis="pauli", data=T))
            free += [int(q) for q in rng.choice(qs, size=free_per_patch, replace=False)]
    free = sorted(free)
    fixed_q = [q for q in range(n) if q not in set(free)]
    fixed_v = [int(v) for v in rng.integers(0, 2, size=len(fixed_q))]
    net = Network(n=n, cuts=cuts, tensors=tensors)
    net.meta.update(name="grid10x12_12patch_40cut_2^24", fixed_qubits=fixed_q, fixed_values=fixed_v,
                    free_qubits=free)
    return net


def random_contraction_order(rng, spec, fixed, temperature=2.0):
    """A randomized greedy contraction order: among pairs of nodes sharing a
    cut, pick the one whose result has the fewest index bits plus Gumbel noise
    (node ids grow as in the plan API: the result of step s is node m + s)."""
    m = len(spec.tensors)
    cuts = {i: set(t.cut_ids) for i, t in enumerate(spec.tensors)}
    outs = {i: sum(1 for q in t.outputs if q not in fixed) for i, t in enumerate(spec.tensors)}
    order, nid = [], m
    while len(cuts) > 1:
        best, pick = None, None
        for a in cuts:
            for b in cuts:
                if a < b and cuts[a] & cuts[b]:
                    bits = 2 * len(cuts[a] ^ cuts[b]) + outs[a] + outs[b]
                    score = bits + temperature * rng.gumbel()
                    if best is None or score < best:
                        best, pick = score, (a, b)
        a, b = pick
        order.append((a, b))
        cuts[nid] = cuts.pop(a) ^ cuts.pop(b)
        outs[nid] = outs.pop(a) + outs.pop(b)
        nid += 1
    return order
