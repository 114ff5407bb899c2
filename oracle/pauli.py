"""Measured subcircuit variants -> Pauli-basis tensors (Sec. II-A).

Readings of the paper used here (the paper says only that the Pauli bases are
"linear combinations" of the measured/initialised variants):

* Pauli digit order I=0, X=1, Y=2, Z=3.
* Upstream (measured) end of a cut, Pauli sigma: use the Z-basis variant for
  sigma in {I, Z}, the X-basis variant for X and the Y-basis variant for Y,
  and sum over the measured cut bit b with weight 1 for I and (-1)^b for
  X, Y, Z (an expectation value of the Pauli observable).
* Downstream (initialised) end: I = rho(0) + rho(1), Z = rho(0) - rho(1),
  X = 2 rho(+) - rho(0) - rho(1), Y = 2 rho(i) - rho(0) - rho(1), applied to
  the measured vectors of the four preparations.
* The factor 1/2 per cut of the identity-channel decomposition is NOT folded
  in here; the reconstruction multiplies by 2^-K once.

Raw layout: see ``workloads.cutting`` (rows mixed radix 3/4 over the local
cuts, first cut slowest; columns x * 2^u + b).  Output layout: rows
sum_t sigma_t * 4^(c-1-t) over the local cuts, columns x.
"""
from __future__ import annotations

import itertools

import numpy as np

# measurement setting used for each Pauli on the upstream side: 0=Z, 1=X, 2=Y
MEAS_FOR_PAULI = {0: 0, 1: 1, 2: 2, 3: 0}
# downstream coefficients over the preparations (|0>, |1>, |+>, |i>)
INIT_COEF = {
    0: (1.0, 1.0, 0.0, 0.0),    # I
    1: (-1.0, -1.0, 2.0, 0.0),  # X
    2: (-1.0, -1.0, 0.0, 2.0),  # Y
    3: (1.0, -1.0, 0.0, 0.0),   # Z
}


def to_pauli(raw: np.ndarray, roles: list, num_outputs: int) -> np.ndarray:
    """Transform one raw tensor.

    roles[t] is 'up' (this subcircuit measures cut t) or 'down' (it prepares
    cut t), in local cut order.  Returns float64 [4^c, 2^o].
    """
    c = len(roles)
    up_idx = [t for t in range(c) if roles[t] == "up"]
    u = len(up_idx)
    radix = [3 if r == "up" else 4 for r in roles]
    weights = [0] * c
    acc = 1
    for t in reversed(range(c)):
        weights[t] = acc
        acc *= radix[t]
    o = num_outputs
    assert raw.shape == (acc, 1 << (o + u)), (raw.shape, acc, o, u)
    # columns as [x][b]
    R = raw.reshape(acc, 1 << o, 1 << u)
    out = np.zeros((4 ** c, 1 << o), dtype=np.float64)
    b = np.arange(1 << u)
    for sigma in itertools.product(range(4), repeat=c):
        row_out = 0
        for t in range(c):
            row_out = row_out * 4 + sigma[t]
        # sign vector over the measured cut bits b
        sign = np.ones(1 << u)
        for i, t in enumerate(up_idx):
            if sigma[t] != 0:
                sign = sign * np.where((b >> i) & 1, -1.0, 1.0)
        # sum over the preparations of the downstream cuts with nonzero weight
        choices = []
        for t in range(c):
            if roles[t] == "up":
                choices.append([(MEAS_FOR_PAULI[sigma[t]], 1.0)])
            else:
                choices.append([(s, w) for s, w in enumerate(INIT_COEF[sigma[t]]) if w != 0.0])
        total = np.zeros(1 << o)
        for combo in itertools.product(*choices):
            coef = 1.0
            row_in = 0
            for t, (dig, w) in enumerate(combo):
                coef *= w
                row_in += dig * weights[t]
            total += coef * (R[row_in] @ sign)
        out[row_out] = total
    return out


def network_pauli_tensors(net):
    """[(cut_ids, outputs, T[4^c, 2^o])] for every tensor of a Network."""
    res = []
    for j, t in enumerate(net.tensors):
        if t.basis == "pauli":
            T = np.asarray(t.data, dtype=np.float64)
        else:
            roles = [net.role(j, c) for c in t.cut_ids]
            T = to_pauli(np.asarray(t.data, dtype=np.float64), roles, len(t.outputs))
        res.append((list(t.cut_ids), list(t.outputs), T))
    return res
