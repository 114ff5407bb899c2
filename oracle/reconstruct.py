"""Reconstruction of output probabilities from Pauli-basis subcircuit tensors.

Definition (Eq. (1), with the 1/2 per cut of the identity-channel
decomposition written out; the paper's formula leaves it implicit):

    P(x) = 2^-K * sum_{sigma in {I,X,Y,Z}^K} prod_j T_j[sigma|E_j, x|O_j]

where E_j are the cuts of subcircuit j (row digits, first local cut slowest)
and O_j its output qubits (bit t of the column <-> qubit outputs[t]).  Output
index convention: bit q of x is the measured value of qubit q.

Two evaluators of that one sum:
  entries_bruteforce          every one of the 4^K terms, summed per entry
  entries_variable_elimination
                              the same multilinear sum with the cut variables
                              summed out one at a time (textbook variable
                              elimination over plain broadcast products); used
                              where 4^K terms per entry are too many, and
                              pinned against the brute force for small K.
"""
from __future__ import annotations

import numpy as np

from .pauli import network_pauli_tensors


def _columns(outputs, xs):
    col = np.zeros(len(xs), dtype=np.int64)
    for t, q in enumerate(outputs):
        col |= ((xs >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << t
    return col


def entries_bruteforce(net, xs, batch=64, tensors=None):
    """P(x) for the global output indices ``xs`` by summing all 4^K terms."""
    xs = np.asarray(xs, dtype=np.uint64)
    tens = tensors if tensors is not None else network_pauli_tensors(net)
    K = net.num_cuts
    S = 4 ** K
    # sigma[s, c]: digit of cut c in assignment s (odometer, cut 0 fastest)
    s = np.arange(S, dtype=np.int64)
    sigma = np.stack([(s >> (2 * c)) & 3 for c in range(K)], axis=1) if K else np.zeros((1, 0), np.int64)
    rows = []
    for cut_ids, _, _ in tens:
        r = np.zeros(S, dtype=np.int64)
        for cid in cut_ids:
            r = r * 4 + sigma[:, cid]
        rows.append(r)
    out = np.empty(len(xs), dtype=np.float64)
    for b0 in range(0, len(xs), batch):
        xb = xs[b0:b0 + batch]
        prod = None
        for (cut_ids, outs, T), r in zip(tens, rows):
            v = T[:, _columns(outs, xb)][r]  # (S, B)
            prod = v if prod is None else prod * v
        out[b0:b0 + batch] = prod.sum(axis=0)
    return out * (0.5 ** K)


def full_distribution(net, **kw):
    return entries_bruteforce(net, np.arange(1 << net.n, dtype=np.uint64), **kw)


def min_degree_order(tensor_cuts, K):
    """Greedy elimination order over the cut variables: always eliminate the
    variable whose merged factor has the fewest variables."""
    factors = [set(c) for c in tensor_cuts]
    order = []
    remaining = set(range(K))
    while remaining:
        best = None
        for v in sorted(remaining):
            merged = set()
            for f in factors:
                if v in f:
                    merged |= f
            size = len(merged)
            if best is None or size < best[0]:
                best = (size, v)
        v = best[1]
        merged = set()
        keep = []
        for f in factors:
            if v in f:
                merged |= f
            else:
                keep.append(f)
        merged.discard(v)
        keep.append(merged)
        factors = keep
        order.append(v)
        remaining.discard(v)
    return order


def _expand(vars_f, arr, union):
    """Broadcast a factor (leading batch axis) to the axis order ``union``."""
    perm = [0] + [1 + vars_f.index(v) for v in union if v in vars_f]
    a = np.transpose(arr, perm)
    shape = [a.shape[0]] + [4 if v in vars_f else 1 for v in union]
    return a.reshape(shape)


def entries_variable_elimination(net, xs, batch=32, tensors=None, order=None):
    """P(x) for ``xs``: per entry, fix the outputs and sum the cut variables
    out one at a time."""
    xs = np.asarray(xs, dtype=np.uint64)
    tens = tensors if tensors is not None else network_pauli_tensors(net)
    K = net.num_cuts
    if order is None:
        order = min_degree_order([c for c, _, _ in tens], K)
    out = np.empty(len(xs), dtype=np.float64)
    for b0 in range(0, len(xs), batch):
        xb = xs[b0:b0 + batch]
        B = len(xb)
        factors = []
        for cut_ids, outs, T in tens:
            v = T[:, _columns(outs, xb)].T  # (B, 4^c)
            factors.append((list(cut_ids), v.reshape([B] + [4] * len(cut_ids))))
        for var in order:
            inv = [f for f in factors if var in f[0]]
            rest = [f for f in factors if var not in f[0]]
            union = []
            for fv, _ in inv:
                for u in fv:
                    if u not in union:
                        union.append(u)
            prod = None
            for fv, arr in inv:
                e = _expand(fv, arr, union)
                prod = e if prod is None else prod * e
            ax = 1 + union.index(var)
            summed = prod.sum(axis=ax)
            union.remove(var)
            rest.append((union, summed))
            factors = rest
        res = np.ones(B)
        for fv, arr in factors:
            assert not fv
            res = res * arr
        out[b0:b0 + B] = res
    return out * (0.5 ** K)


def restrict_fixed(net, fixed, tensors=None):
    """Pauli-basis tensors of ``net`` with the qubits in ``fixed`` (qubit ->
    bit) held at their values: each tensor keeps the columns that agree with
    them, and the remaining outputs are renumbered by rank among the free
    qubits (ascending).  Evaluating Eq. (1) on the result at y gives P(x) for
    the x that agrees with ``fixed`` and carries y on the free qubits, so
    global indices wider than 64 bits never have to be formed.  Returns
    (tensors, number of free qubits)."""
    tens = tensors if tensors is not None else network_pauli_tensors(net)
    free = [q for q in range(net.n) if q not in fixed]
    rank = {q: i for i, q in enumerate(free)}
    out = []
    for cut_ids, outs, T in tens:
        keep = [t for t, q in enumerate(outs) if q not in fixed]
        base = 0
        for t, q in enumerate(outs):
            if q in fixed:
                base |= int(fixed[q]) << t
        cols = np.full(1 << len(keep), base, dtype=np.int64)
        y = np.arange(1 << len(keep), dtype=np.int64)
        for i, t in enumerate(keep):
            cols |= ((y >> i) & 1) << t
        out.append((list(cut_ids), [rank[outs[t]] for t in keep], T[:, cols]))
    return out, len(free)
