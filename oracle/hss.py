"""Heavy State Selection (Sec. IV, Alg. 1) and its metrics (Eqs. (9)-(13)).

TEST INFRASTRUCTURE ONLY (see the package header).

Alg. 1 in the paper's order, on the Pauli-basis subcircuit tensors T_j (the
subcircuit outputs p_j^e of Eq. (1): row = edge permutation e, column =
binary state i of the subcircuit's output qubits):

  1. per subcircuit j and state i, the L2 norm over all edge permutations,
     ||p_{j,i}|| = sqrt(sum_e (p_{j,i}^e)^2);
  2. every subcircuit starts with its heaviest state (ties: smaller i);
  3. the other (j, i) are sorted by norm, descending (ties: smaller j, then
     smaller i);
  4. while the product of the subset sizes is below s_max, the next (j, i)
     is popped and i joins subcircuit j's subset.

Readings: the norms are taken over the Pauli-basis rows (the p_j^e of
Eq. (1)); the loop stops at the first product >= s_max, so the product may
exceed s_max (the loop condition as stated); the retained output states are
the product set x_1 x ... x x_m.
"""
from __future__ import annotations

import numpy as np

from .pauli import network_pauli_tensors


def column_norms(T):
    """||p_{j,i}|| for every column i of one tensor (float64)."""
    T = np.asarray(T, dtype=np.float64)
    return np.sqrt((T * T).sum(axis=0))


def select(norms, s_max):
    """Alg. 1 on per-tensor norm vectors; returns each subset, ascending."""
    chosen = []
    rest = []
    for j, nv in enumerate(norms):
        first = int(np.argmax(nv))  # argmax returns the smallest index of ties
        chosen.append({first})
        for i, v in enumerate(nv):
            if i != first:
                rest.append((-float(v), j, i))
    rest.sort()
    size = 1
    for c in chosen:
        size *= len(c)
    pos = 0
    while size < s_max and pos < len(rest):
        _, j, i = rest[pos]
        pos += 1
        size = size // len(chosen[j]) * (len(chosen[j]) + 1)
        chosen[j].add(i)
    return [np.array(sorted(c), dtype=np.int64) for c in chosen]


def heavy_states(net, s_max, tensors=None):
    """(subsets, norms) of the network's subcircuits."""
    tens = tensors if tensors is not None else network_pauli_tensors(net)
    norms = [column_norms(T) for _, _, T in tens]
    return select(norms, s_max), norms


def product_indices(net, subsets, tensors=None):
    """Global output indices of the retained product states, tensor 0's
    subset index fastest: entry c = sum_j y_j * prod_{l<j} |x_l| is the state
    whose qubits of tensor j carry the bits of x_j[y_j]."""
    tens = tensors if tensors is not None else network_pauli_tensors(net)
    total = 1
    for s in subsets:
        total *= len(s)
    c = np.arange(total, dtype=np.int64)
    xs = np.zeros(total, dtype=np.uint64)
    for (cut_ids, outs, _), s in zip(tens, subsets):
        y = c % len(s)
        c = c // len(s)
        col = s[y]
        for t, q in enumerate(outs):
            xs |= ((col >> t) & 1).astype(np.uint64) << np.uint64(q)
    return xs


def metrics(p_selected, p_full, n):
    """Eqs. (9)-(13): P_HSS, P_HSS^max (sum of the |HSS| largest true
    probabilities), r_P = P_HSS / P_HSS^max, r_|HSS| = |HSS| / 2^n and
    eta = P_HSS / r_|HSS|."""
    size = len(p_selected)
    p_hss = float(np.sum(p_selected))
    p_max = float(np.sort(np.asarray(p_full))[::-1][:size].sum())
    r_size = size / float(2 ** n)
    return {"P_HSS": p_hss, "P_HSS_max": p_max, "r_P": p_hss / p_max if p_max else 0.0,
            "r_size": r_size, "eta": p_hss / r_size}
