"""Multiplication count of a pairwise contraction sequence (Sec. III-C).

Contracting two tensors costs the product of the dimensions of every index
either of them carries (shared cut indices, open cut indices and, when
counted, output bits): dim 4 per cut, 2 per output qubit.  The brute-force
method of prior work costs 4^K * (m - 1) multiplications per output state
(Eq. (5)).
"""
from __future__ import annotations


def sequence_cost(tensor_cuts, tensor_outputs, sequence, count_outputs=True):
    """tensor_cuts[j]: set of cut ids of tensor j; sequence: list of (a, b)
    pairs of tensor ids, each step creating a new id (SSA, appended).
    Returns the per-step multiplication counts."""
    cuts = [set(c) for c in tensor_cuts]
    outs = [int(o) for o in tensor_outputs]
    steps = []
    for a, b in sequence:
        union = cuts[a] | cuts[b]
        cost = 4 ** len(union)
        if count_outputs:
            cost *= 2 ** (outs[a] + outs[b])
        steps.append(cost)
        cuts.append(cuts[a] ^ cuts[b])
        outs.append(outs[a] + outs[b])
    return steps


def bruteforce_cost(num_cuts, num_tensors):
    return 4 ** num_cuts * (num_tensors - 1)
