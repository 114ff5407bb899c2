"""Seeded batch of uneven reconstructions for batched execution.

Job i draws, from its own seed stream: n uniform in 16..28 qubits, m uniform
in 2..5 subcircuits, a cut target uniform in 2..10, a layout (a line, or a
near-square grid filled row by row) and a depth uniform in 4..8.  Each layer
is a random Rx/Ry/Rz rotation (angle uniform in [0, 2 pi)) on every qubit
followed by CZ on one brickwork class of nearest-neighbour bonds.  The qubits
form m contiguous groups in index order, one subcircuit each.  A CZ whose
qubits lie in different groups belongs to one of the two (seeded coin); the
other wire is cut into that subcircuit and, at its next rotation, cut back.
Cross-group CZs are kept only while the cut count (including the pending
returns) stays within the target.  Subcircuit tensors are exact (statevector
simulation of every measured variant, Sec. II-A).

Generation is bounded: an instance whose simulation cost (sum over
subcircuits of 4^d (gates + 3^u) 2^width amplitude updates), raw or
Pauli-basis tensor size, or estimated contraction work (greedy pairwise
order) exceeds the caps below is redrawn with a lower cut target, keeping n,
m and the layout; so large-n jobs lean toward fewer cuts.  describe()
reports the accepted distribution."""
from __future__ import annotations

import numpy as np

from .circuit import Circuit
from .configs import rng_for
from .cutting import cut_circuit, cut_shapes

CONFIG = 4
N_RANGE = (16, 28)
M_RANGE = (2, 5)
K_RANGE = (2, 10)
DEPTH_RANGE = (4, 8)
SIM_CAP = 1 << 27          # amplitude updates to build one job's tensors
TENSOR_CAP = 1 << 25       # entries of one raw or Pauli-basis tensor
FLOP_CAP = float(1 << 38)  # estimated contraction flops of one job
INTER_CAP = 1 << 29        # entries of the largest intermediate


def _bonds(n, layout):
    """Brickwork bond classes of nearest-neighbour pairs."""
    if layout == "line":
        return [[(q, q + 1) for q in range(s, n - 1, 2)] for s in (0, 1)]
    rows = int(np.floor(np.sqrt(n)))
    cols = -(-n // rows)
    at = lambda r, c: r * cols + c
    classes = []
    for s in (0, 1):
        classes.append([(at(r, c), at(r, c + 1)) for r in range(rows) for c in range(s, cols - 1, 2)
                        if at(r, c + 1) < n])
    for s in (0, 1):
        classes.append([(at(r, c), at(r + 1, c)) for r in range(s, rows - 1, 2) for c in range(cols)
                        if at(r + 1, c) < n])
    return classes


def _circuit(n, m, layout, depth, target, rng):
    home = [q * m // n for q in range(n)]
    c = Circuit(n)
    sub = []
    owner = list(home)
    cuts = 0
    classes = _bonds(n, layout)
    for layer in range(depth):
        for q in range(n):
            c.add(("rx", "ry", "rz")[rng.integers(3)], q, params=(rng.uniform(0, 2 * np.pi),))
            sub.append(home[q])
            if owner[q] != home[q]:
                cuts += 1
                owner[q] = home[q]
        for a, b in classes[layer % len(classes)]:
            if home[a] == home[b]:
                c.add("cz", a, b)
                sub.append(home[a])
                continue
            own = home[a] if rng.integers(2) else home[b]
            new = int(owner[a] != own) + int(owner[b] != own)
            away = sum(owner[q] != home[q] for q in range(n) if q not in (a, b))
            away += int(own != home[a]) + int(own != home[b])
            pending = away if layer < depth - 1 else 0
            if cuts + new + pending > target:
                continue
            c.add("cz", a, b)
            sub.append(own)
            cuts += new
            owner[a] = owner[b] = own
    return c, sub, home


def contraction_estimate(cuts, outputs):
    """Greedy pairwise contraction (smallest result first): (flops, largest
    intermediate entries).  An upper bound on what a good order costs."""
    live = {j: (outputs[j], {c for c, e in enumerate(cuts) if j in e}) for j in range(len(outputs))}
    flops, largest = 0.0, 0
    while len(live) > 1:
        best = None
        keys = sorted(live)
        for i, a in enumerate(keys):
            for b in keys[i + 1:]:
                oa, ca = live[a]
                ob, cb = live[b]
                shared = ca & cb
                if not shared and len(live) > 2 and any(live[x][1] & ca for x in keys if x != a):
                    continue
                open_ = (ca | cb) - shared
                size = 2 ** (oa + ob) * 4 ** len(open_)
                f = 2.0 * size * 4 ** len(shared)
                if best is None or (size, f) < (best[0], best[1]):
                    best = (size, f, a, b, oa + ob, open_)
        size, f, a, b, o, open_ = best
        flops += f
        largest = max(largest, size)
        del live[b]
        live[a] = (o, open_)
    return flops, largest


def _accept(cuts, shapes):
    sim = sum(4 ** s["d"] * (s["gates"] + 3 ** s["u"]) * 2 ** s["width"] for s in shapes)
    if sim > SIM_CAP:
        return False
    for s in shapes:
        if 4 ** s["d"] * 3 ** s["u"] * 2 ** s["width"] > TENSOR_CAP:
            return False
        if 4 ** (s["d"] + s["u"]) * 2 ** s["outputs"] > TENSOR_CAP:
            return False
    flops, largest = contraction_estimate(cuts, [s["outputs"] for s in shapes])
    return flops <= FLOP_CAP and largest <= INTER_CAP


def draw(i, seed=None):
    """The (n, m, layout, depth, circuit, gate owners, homes) of job i."""
    rng = rng_for(CONFIG, i, seed)
    n = int(rng.integers(N_RANGE[0], N_RANGE[1] + 1))
    m = int(rng.integers(M_RANGE[0], M_RANGE[1] + 1))
    layout = ("line", "grid")[int(rng.integers(2))]
    target = int(rng.integers(K_RANGE[0], K_RANGE[1] + 1))
    while True:
        depth = int(rng.integers(DEPTH_RANGE[0], DEPTH_RANGE[1] + 1))
        circ, sub, home = _circuit(n, m, layout, depth, target, rng)
        cuts, shapes = cut_shapes(circ, sub, num_subs=m, idle_sub=home)
        if len(cuts) >= K_RANGE[0] and all(s["width"] > 0 for s in shapes) and _accept(cuts, shapes):
            return n, m, layout, depth, circ, sub, home, target
        # too few cuts: try another circuit; too costly: lower the target
        if len(cuts) >= K_RANGE[0]:
            target = max(K_RANGE[0], target - 1)


def job(i, seed=None):
    """Network of job i (exact raw subcircuit tensors)."""
    n, m, layout, depth, circ, sub, home, target = draw(i, seed)
    net = cut_circuit(circ, sub, num_subs=m, idle_sub=home)
    net.meta.update(circuit=circ, name=f"batch{i}_n{n}_m{m}_{layout}_d{depth}", layout=layout,
                    depth=depth, target=target)
    return net


def describe(nets):
    """Accepted distribution of a list of jobs."""
    ns = np.array([x.n for x in nets])
    ms = np.array([len(x.tensors) for x in nets])
    ks = np.array([x.num_cuts for x in nets])
    return {
        "jobs": len(nets),
        "n_hist": {int(v): int((ns == v).sum()) for v in np.unique(ns)},
        "m_hist": {int(v): int((ms == v).sum()) for v in np.unique(ms)},
        "k_hist": {int(v): int((ks == v).sum()) for v in np.unique(ks)},
        "layouts": {l: int(sum(x.meta.get("layout") == l for x in nets)) for l in ("line", "grid")},
        "output_bytes_f32": int(sum(4 << x.n for x in nets)),
    }
