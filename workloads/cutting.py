"""Wire cutting of a gate-list circuit into subcircuits, and the measured
subcircuit variants (the quantum half of the method, Sec. II-A).

A cut on a qubit wire splits it into an upstream segment, whose end is
measured in one of the Z, X, Y bases (I shares the Z rotation), and a
downstream segment, which starts in one of |0>, |1>, |+>, |i>.  Running every
combination of those settings gives 3^u * 4^d probability vectors per
subcircuit (the variant count of Eq. (6)).  This module only produces those
measured vectors ("raw" tensors); turning them into Pauli-basis tensors is the
reconstruction's job and lives elsewhere.

Raw tensor layout for subcircuit j (float64, 2-D):
  rows: mixed-radix digits over j's cuts in its local cut order, first cut the
        slowest digit; radix 3 where j is the upstream end (0=Z, 1=X, 2=Y
        measurement), radix 4 where j is the downstream end (0=|0>, 1=|1>,
        2=|+>, 3=|i> initialisation);
  cols: x * 2^u + b, where bit t of x is the measured value of output qubit
        outputs[t] and bit i of b is the measured value of the i-th upstream
        cut in local cut order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuit import Circuit, Gate, apply_1q, apply_gate, ONE_QUBIT

_H = ONE_QUBIT["h"]()
_SDG = ONE_QUBIT["sdg"]()
_SQ2 = 1.0 / np.sqrt(2.0)
# single-qubit initial states for downstream cut digits 0..3
INIT_STATES = [
    np.array([1, 0], dtype=np.complex128),
    np.array([0, 1], dtype=np.complex128),
    np.array([_SQ2, _SQ2], dtype=np.complex128),
    np.array([_SQ2, 1j * _SQ2], dtype=np.complex128),
]


@dataclass
class TensorSpec:
    cut_ids: list            # local cut order (first = slowest row digit)
    outputs: list            # bit t of the column index <-> global qubit outputs[t]
    basis: str               # "raw" or "pauli"
    data: np.ndarray         # float64, 2-D

    @property
    def rows(self):
        return self.data.shape[0]


@dataclass
class Network:
    n: int                   # qubits of the uncut circuit
    cuts: list               # cuts[c] = (upstream tensor, downstream tensor)
    tensors: list            # TensorSpec per subcircuit
    meta: dict = field(default_factory=dict)

    @property
    def num_cuts(self):
        return len(self.cuts)

    def role(self, j, c):
        """'up' if tensor j is the measured (upstream) end of cut c, else 'down'."""
        up, down = self.cuts[c]
        if up == j:
            return "up"
        assert down == j
        return "down"


def _segments(circ: Circuit, gate_sub, idle_sub):
    """Split each wire into maximal runs of gates owned by one subcircuit."""
    segs = []  # (qubit, sub, [gate indices])
    per_q = [[] for _ in range(circ.n)]
    for gi, g in enumerate(circ.gates):
        for q in g.qubits:
            per_q[q].append(gi)
    for q in range(circ.n):
        tl = per_q[q]
        if not tl:
            segs.append([q, idle_sub[q], []])
            continue
        cur = [q, gate_sub[tl[0]], [tl[0]]]
        for gi in tl[1:]:
            if gate_sub[gi] == cur[1]:
                cur[2].append(gi)
            else:
                segs.append(cur)
                cur = [q, gate_sub[gi], [gi]]
        segs.append(cur)
    return segs


def cut_circuit(circ: Circuit, gate_sub, num_subs=None, idle_sub=None):
    """Cut `circ` where consecutive gates of a wire belong to different subcircuits.

    gate_sub[g] is the subcircuit owning gate g.  Wires without gates go to
    idle_sub[q] (default subcircuit 0).  Returns (Network with raw tensors,
    per-subcircuit info dict).
    """
    n = circ.n
    if idle_sub is None:
        idle_sub = [0] * n
    if num_subs is None:
        num_subs = max(list(gate_sub) + list(idle_sub)) + 1
    segs = _segments(circ, gate_sub, idle_sub)
    # index segments per qubit in wire order
    by_q = [[] for _ in range(n)]
    for si, s in enumerate(segs):
        by_q[s[0]].append(si)
    cuts = []          # (up sub, down sub)
    seg_start_cut = {}  # seg -> cut id entering it
    seg_end_cut = {}    # seg -> cut id leaving it
    for q in range(n):
        chain = by_q[q]
        for a, b in zip(chain[:-1], chain[1:]):
            cid = len(cuts)
            cuts.append((segs[a][1], segs[b][1]))
            seg_end_cut[a] = cid
            seg_start_cut[b] = cid
    tensors = []
    infos = []
    for j in range(num_subs):
        my = [si for si in range(len(segs)) if segs[si][1] == j]
        local = {si: l for l, si in enumerate(my)}
        w = len(my)
        my_cuts = sorted({seg_start_cut[si] for si in my if si in seg_start_cut}
                         | {seg_end_cut[si] for si in my if si in seg_end_cut})
        up_cuts = [c for c in my_cuts if cuts[c][0] == j]
        outputs = sorted(segs[si][0] for si in my if si not in seg_end_cut)
        out_local = {segs[si][0]: local[si] for si in my if si not in seg_end_cut}
        cut_local = {}
        for si in my:
            if si in seg_start_cut:
                cut_local[("down", seg_start_cut[si])] = local[si]
            if si in seg_end_cut:
                cut_local[("up", seg_end_cut[si])] = local[si]
        # gates of this subcircuit, mapped to local qubits (segment active at that gate)
        gate_local = []
        for gi, g in enumerate(circ.gates):
            if gate_sub[gi] != j:
                continue
            qm = {}
            for q in g.qubits:
                owner = [si for si in by_q[q] if gi in segs[si][2]]
                assert len(owner) == 1 and segs[owner[0]][1] == j
                qm[q] = local[owner[0]]
            gate_local.append(Gate(g.name, tuple(qm[q] for q in g.qubits), g.params))
        radices = [3 if cuts[c][0] == j else 4 for c in my_cuts]
        u = len(up_cuts)
        o = len(outputs)
        nrows = int(np.prod(radices)) if radices else 1
        data = np.zeros((nrows, 1 << (o + u)), dtype=np.float64)
        # column gather: local prob index -> column
        li = np.arange(1 << w, dtype=np.int64)
        col = np.zeros(1 << w, dtype=np.int64)
        for t, q in enumerate(outputs):
            col |= ((li >> out_local[q]) & 1) << (u + t)
        for i, c in enumerate(up_cuts):
            col |= ((li >> cut_local[("up", c)]) & 1) << i
        down_cuts = [c for c in my_cuts if cuts[c][1] == j]
        # row index of a digit assignment: mixed radix, first cut slowest
        weights = {}
        acc = 1
        for c, rad in zip(reversed(my_cuts), reversed(radices)):
            weights[c] = acc
            acc *= rad
        for init in np.ndindex(*([4] * len(down_cuts))):
            dig = dict(zip(down_cuts, init))
            # product initial state; local qubit l is bit l (kron puts its
            # second factor in the low bits)
            states = []
            for l in range(w):
                si = my[l]
                if si in seg_start_cut:
                    states.append(INIT_STATES[dig[seg_start_cut[si]]])
                else:
                    states.append(INIT_STATES[0])
            psi0 = states[w - 1] if w else np.ones(1, dtype=np.complex128)
            for l in range(w - 2, -1, -1):
                psi0 = np.kron(psi0, states[l])
            for g in gate_local:
                psi0 = apply_gate(psi0, w, g)
            for meas in np.ndindex(*([3] * len(up_cuts))):
                psi = psi0
                for c, m in zip(up_cuts, meas):
                    l = cut_local[("up", c)]
                    if m == 1:
                        psi = apply_1q(psi, w, l, _H)
                    elif m == 2:
                        psi = apply_1q(apply_1q(psi, w, l, _SDG), w, l, _H)
                p = psi.real ** 2 + psi.imag ** 2
                r = sum(weights[c] * d for c, d in zip(down_cuts, init))
                r += sum(weights[c] * m for c, m in zip(up_cuts, meas))
                # every local qubit is either an output or an upstream cut
                # end, so col is a bijection
                data[r, col] = p
        tensors.append(TensorSpec(cut_ids=my_cuts, outputs=outputs, basis="raw", data=data))
        infos.append({"width": w, "u": u, "d": len(my_cuts) - u, "outputs": o})
    net = Network(n=n, cuts=cuts, tensors=tensors, meta={"subcircuits": infos})
    return net


def cut_shapes(circ: Circuit, gate_sub, num_subs=None, idle_sub=None):
    """The cut list and per-subcircuit sizes cut_circuit would produce, without
    simulating anything: (cuts, [{"width", "u", "d", "outputs", "gates"}]).
    Lets a generator bound simulation cost and tensor sizes up front."""
    n = circ.n
    if idle_sub is None:
        idle_sub = [0] * n
    if num_subs is None:
        num_subs = max(list(gate_sub) + list(idle_sub)) + 1
    segs = _segments(circ, gate_sub, idle_sub)
    by_q = [[] for _ in range(n)]
    for si, s in enumerate(segs):
        by_q[s[0]].append(si)
    cuts, starts, ends = [], set(), set()
    for q in range(n):
        chain = by_q[q]
        for a, b in zip(chain[:-1], chain[1:]):
            cuts.append((segs[a][1], segs[b][1]))
            ends.add(a)
            starts.add(b)
    shapes = []
    for j in range(num_subs):
        my = [si for si in range(len(segs)) if segs[si][1] == j]
        u = sum(si in ends for si in my)
        shapes.append({"width": len(my), "u": u, "d": sum(si in starts for si in my),
                       "outputs": len(my) - u, "gates": sum(1 for g in gate_sub if g == j)})
    return cuts, shapes


def assign_from_partition(circ: Circuit, labels):
    """Subcircuit of every gate from a partition of the two-qubit gates
    (labels: gate index -> partition): a single-qubit gate joins the next
    two-qubit gate on its wire, else the previous one; a wire without
    two-qubit gates belongs to partition 0.  Returns (gate_sub, idle_sub,
    number of partitions) for cut_circuit."""
    n = circ.n
    two = [[] for _ in range(n)]
    for g, gate in enumerate(circ.gates):
        if len(gate.qubits) == 2:
            for q in gate.qubits:
                two[q].append(g)
    gate_sub = []
    for g, gate in enumerate(circ.gates):
        if len(gate.qubits) == 2:
            gate_sub.append(int(labels[g]))
            continue
        q = gate.qubits[0]
        nxt = [h for h in two[q] if h > g]
        prv = [h for h in two[q] if h < g]
        gate_sub.append(int(labels[nxt[0]]) if nxt else (int(labels[prv[-1]]) if prv else 0))
    idle = [int(labels[two[q][0]]) if two[q] else 0 for q in range(n)]
    parts = max(list(labels.values()) + [0]) + 1
    return gate_sub, idle, parts
