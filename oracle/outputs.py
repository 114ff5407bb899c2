"""Output forms of a reconstructed probability vector.

* top-k: the k largest entries, larger value first, equal values by smaller
  index; the sum of the top |HSS| true probabilities is P_HSS^max (Eq. (10)).
* marginal: probabilities of the kept qubits, summing the others out; with no
  kept qubit it is the total probability (1 for a physical circuit).
"""
from __future__ import annotations

import numpy as np


def topk(p, k):
    p = np.asarray(p)
    idx = np.arange(len(p), dtype=np.int64)
    order = np.lexsort((idx, -p.astype(np.float64)))
    sel = order[:k]
    return sel, p[sel].astype(np.float64)


def marginal(p, n, keep):
    """out[y], bit i of y <-> qubit keep[i]; float64 sums."""
    p = np.asarray(p, dtype=np.float64).reshape([2] * n)  # axis a <-> qubit n-1-a
    drop_axes = tuple(n - 1 - q for q in range(n) if q not in keep)
    m = p.sum(axis=drop_axes) if drop_axes else p
    # remaining axes are kept qubits in descending qubit order
    remaining = sorted(keep, reverse=True)
    # want axis order: keep[-1] ... keep[0] (so that keep[0] is the lowest bit)
    perm = [remaining.index(q) for q in reversed(keep)]
    m = np.transpose(m, perm) if perm else m
    return np.asarray(m).reshape(-1)
