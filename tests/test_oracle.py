"""Pins of the CPU oracle against facts fixed by the paper and by physics,
independent of the oracle's own formulas:

* the uncut circuit's statevector (the reconstruction must reproduce it);
* closed forms of GHZ, W-state and AQFT outputs (Sec. VII-B);
* normalisation of measured/prepared variants (sums over a tensor's columns);
* planted mistakes (a flipped Y sign, a dropped 1/2 per cut, X/Y swapped)
  must be caught by the statevector pin;
* variable elimination against the brute-force sum, and the two-tensor case
  against a plain matrix product;
* the worked cost example of Sec. III-C (golden fixture).
"""
import itertools
import os

import numpy as np
import pytest

from oracle import outputs as oout
from oracle import plancost
from oracle.pauli import network_pauli_tensors
from oracle.reconstruct import (entries_bruteforce, entries_variable_elimination,
                                full_distribution)
from workloads import configs, probabilities, synthetic
from workloads.circuit import Circuit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_simulator_basics():
    c = Circuit(3).add("x", 0)
    assert probabilities(c)[1] == pytest.approx(1.0)
    c = Circuit(2).add("h", 0).add("cx", 0, 1)
    p = probabilities(c)
    assert p == pytest.approx([0.5, 0, 0, 0.5])
    # controlled Ry acts only when the control (first qubit) is 1
    c = Circuit(2).add("cry", 0, 1, params=(np.pi,))
    assert probabilities(c)[0] == pytest.approx(1.0)
    c = Circuit(2).add("x", 0).add("cry", 0, 1, params=(np.pi,))
    assert probabilities(c)[3] == pytest.approx(1.0)


def _statevector_case(net):
    p = probabilities(net.meta["circuit"])
    P = full_distribution(net)
    return np.abs(P - p).max()


@pytest.mark.parametrize("builder", [
    lambda: configs.config1(),
    lambda: configs.ghz(10, 3),
    lambda: configs.w_state(9, 3),
    lambda: configs.aqft(10, 3, 2),
] + [(lambda s=s: configs.random_cut_circuit(9, 3, 4, 3, s)) for s in range(6)])
def test_reconstruction_matches_statevector(builder):
    net = builder()
    assert net.num_cuts >= 1
    assert _statevector_case(net) < 1e-12


def test_config1_structure_and_invariants():
    net = configs.config1()
    assert net.num_cuts == 2
    assert [t.data.shape for t in net.tensors] == [(12, 128), (12, 128)]
    P = full_distribution(net)
    assert abs(P.sum() - 1.0) < 1e-12
    assert P.min() > -1e-15


@pytest.mark.parametrize("n,m", [(12, 4), (14, 3)])
def test_ghz_closed_form(n, m):
    P = full_distribution(configs.ghz(n, m))
    expect = np.zeros(1 << n)
    expect[0] = expect[-1] = 0.5
    assert np.abs(P - expect).max() < 1e-13


@pytest.mark.parametrize("n,m", [(10, 3), (12, 4)])
def test_w_closed_form(n, m):
    P = full_distribution(configs.w_state(n, m))
    expect = np.zeros(1 << n)
    for i in range(n):
        expect[1 << i] = 1.0 / n
    assert np.abs(P - expect).max() < 1e-13


@pytest.mark.parametrize("n,m,d", [(10, 3, 2), (12, 4, 3)])
def test_aqft_closed_form(n, m, d):
    P = full_distribution(configs.aqft(n, m, d))
    assert np.abs(P - 2.0 ** -n).max() < 1e-13


def test_column_sums_of_variants():
    """A subcircuit whose cuts are all prepared (downstream): each preparation
    is a normalised state, so sum_x T[sigma, x] = prod_t (2 if I else 0).
    All measured (upstream): sum_x T[I.., x] = 1 and sum_x T[sigma, x] is the
    Pauli expectation of the cut qubits, bounded by 1 in magnitude."""
    net = configs.ghz(12, 4)
    tens = network_pauli_tensors(net)
    checked_down = checked_up = 0
    for j, (cids, outs, T) in enumerate(tens):
        roles = [net.role(j, c) for c in cids]
        s = T.sum(axis=1)
        if all(r == "down" for r in roles):
            for row, sig in enumerate(itertools.product(range(4), repeat=len(cids))):
                expect = np.prod([2.0 if d == 0 else 0.0 for d in sig])
                assert abs(s[row] - expect) < 1e-12
            checked_down += 1
        if all(r == "up" for r in roles):
            assert abs(s[0] - 1.0) < 1e-12
            assert np.all(np.abs(s) <= 1 + 1e-12)
            checked_up += 1
    assert checked_down >= 1 and checked_up >= 1


def _planted(net, mutate):
    tens = network_pauli_tensors(net)
    tens = [(c, o, T.copy()) for c, o, T in tens]
    mutate(net, tens)
    p = probabilities(net.meta["circuit"])
    P = entries_bruteforce(net, np.arange(1 << net.n, dtype=np.uint64), tensors=tens)
    return np.abs(P - p).max()


def _rows_with_digit(cids, cut, digit):
    t = cids.index(cut)
    c = len(cids)
    return [r for r in range(4 ** c) if (r >> (2 * (c - 1 - t))) & 3 == digit]


def test_planted_mistakes_are_caught():
    net = configs.config1()
    cut = 0
    up = net.cuts[cut][0]

    def flip_up_y(net, tens):
        cids, _, T = tens[up]
        T[_rows_with_digit(cids, cut, 2)] *= -1

    def drop_half(net, tens):
        tens[0][2][:] *= 2.0

    def swap_xy(net, tens):
        cids, _, T = tens[up]
        rx = _rows_with_digit(cids, cut, 1)
        ry = _rows_with_digit(cids, cut, 2)
        T[rx], T[ry] = T[ry].copy(), T[rx].copy()

    for mut in (flip_up_y, drop_half, swap_xy):
        assert _planted(net, mut) > 1e-3, mut.__name__


@pytest.mark.parametrize("seed", range(6))
def test_variable_elimination_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(3, 6))
    K = int(rng.integers(m - 1, 8))
    outs = [int(x) for x in rng.integers(1, 4, size=m)]
    net = synthetic.random_network(m, K, outs, seed=100 + seed)
    xs = np.arange(1 << net.n, dtype=np.uint64)
    a = entries_bruteforce(net, xs)
    b = entries_variable_elimination(net, xs)
    assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(a).max())


def test_two_tensors_is_a_matrix_product():
    net = synthetic.random_network(2, 3, [3, 4], seed=7)
    (ca, oa, A), (cb, ob, B) = network_pauli_tensors(net)
    # reorder B's rows to A's cut order
    perm = []
    for sig in itertools.product(range(4), repeat=len(ca)):
        d = dict(zip(ca, sig))
        r = 0
        for c in cb:
            r = r * 4 + d[c]
        perm.append(r)
    C = (A.T @ B[perm]) * 0.5 ** net.num_cuts  # C[xa, xb]
    P = full_distribution(net)
    for xa in range(1 << len(oa)):
        for xb in range(1 << len(ob)):
            x = 0
            for t, q in enumerate(oa):
                x |= ((xa >> t) & 1) << q
            for t, q in enumerate(ob):
                x |= ((xb >> t) & 1) << q
            assert abs(P[x] - C[xa, xb]) < 1e-15


def test_topk_against_sorting_tuples():
    rng = np.random.default_rng(3)
    p = rng.integers(0, 6, size=300).astype(np.float64) / 7.0  # many ties
    k = 17
    idx, val = oout.topk(p, k)
    ref = sorted(range(len(p)), key=lambda i: (-p[i], i))[:k]
    assert list(idx) == ref
    assert np.array_equal(val, p[ref])


def test_marginal_against_loops():
    rng = np.random.default_rng(4)
    n = 7
    p = rng.random(1 << n)
    keep = [5, 1, 3]
    got = oout.marginal(p, n, keep)
    ref = np.zeros(1 << len(keep))
    for x in range(1 << n):
        y = sum(((x >> q) & 1) << i for i, q in enumerate(keep))
        ref[y] += p[x]
    assert np.abs(got - ref).max() < 1e-14
    assert oout.marginal(p, n, []) == pytest.approx([p.sum()])


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_worked_example_cost():
    rows = _read_golden("worked_example_cost.txt")
    cuts = [set(int(x) for x in r[3:]) for r in rows if r[0] == "tensor"]
    steps = [(int(r[1]), int(r[2]), int(r[4])) for r in rows if r[0] == "step"]
    total = int([r for r in rows if r[0] == "total"][0][1])
    prior = int([r for r in rows if r[0] == "prior"][0][1])
    got = plancost.sequence_cost(cuts, [0] * len(cuts), [(a, b) for a, b, _ in steps],
                                 count_outputs=False)
    assert got == [c for _, _, c in steps]
    assert sum(got) == total
    assert plancost.bruteforce_cost(4, 4) == prior
    # Eq. (4): sum of step costs <= (m-1) 4^Kmax with Kmax = 3 here
    assert sum(got) <= 3 * 4 ** 3


def test_mlp_oracle_gradients_match_finite_differences():
    from oracle import mlp
    F, H = 5, 7
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(mlp.num_params(F, H)) * 0.5
    X = rng.standard_normal((9, F))
    t = rng.standard_normal(9)
    g = mlp.gradients(theta, X, t, F, H)
    eps = 1e-6
    num = np.empty_like(theta)
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        num[i] = (mlp.loss(tp, X, t, F, H) - mlp.loss(tm, X, t, F, H)) / (2 * eps)
    assert np.abs(g - num).max() <= 1e-6 * max(1.0, np.abs(num).max())


def test_mlp_oracle_one_unit_network_by_hand():
    # F = H = 1, theta = (W1, b1, W2, b2, w3, b3) = (0.5, 0.25, -2, 3, 4, -1),
    # worked by hand.  x = 2: z1 = 1.25, z2 = 0.5, y = 4 * 0.5 - 1 = 1; with
    # t = 0.25, L = 0.75^2 and dL/dy = 1.5, so dw3 = 0.5 * 1.5, db3 = 1.5,
    # dz2 = 1.5 * 4 = 6, dW2 = 1.25 * 6, db2 = 6, dz1 = 6 * -2 = -12,
    # dW1 = 2 * -12, db1 = -12.
    from oracle import mlp
    theta = np.array([0.5, 0.25, -2.0, 3.0, 4.0, -1.0])
    y, _ = mlp.forward(theta, [[2.0]], 1, 1)
    assert y.tolist() == [1.0]
    assert mlp.loss(theta, [[2.0]], [0.25], 1, 1) == 0.5625
    assert mlp.gradients(theta, [[2.0]], [0.25], 1, 1).tolist() == [-24.0, -12.0, 7.5, 6.0, 0.75, 1.5]
    # x = -2: z1 = -0.75 is cut by the first ReLU, z2 = 3, y = 11 (without
    # that ReLU: 17); with t = 0, dL/dy = 22: dw3 = 66, db3 = 22, db2 = 88,
    # and nothing flows into the first layer or W2 (h1 = 0)
    y, _ = mlp.forward(theta, [[-2.0]], 1, 1)
    assert y.tolist() == [11.0]
    assert mlp.gradients(theta, [[-2.0]], [0.0], 1, 1).tolist() == [0.0, 0.0, 0.0, 88.0, 66.0, 22.0]
    # the batch mean: both samples together halve and add the two gradients
    g2 = mlp.gradients(theta, [[2.0], [-2.0]], [0.25, 0.0], 1, 1)
    assert g2.tolist() == [-12.0, -6.0, 3.75, 47.0, 33.375, 11.75]


def test_restrict_fixed_equals_entries_of_the_full_distribution():
    # a fixed-qubit slice read off the full vector, entry by entry
    from oracle.reconstruct import restrict_fixed
    spec = synthetic.random_network(4, 6, [3, 4, 2, 3], seed=91)
    full = full_distribution(spec)
    fixed = {1: 1, 4: 0, 7: 1, 11: 0}
    tens, nfree = restrict_fixed(spec, fixed)
    assert nfree == spec.n - len(fixed)
    free = [q for q in range(spec.n) if q not in fixed]
    ys = np.arange(1 << nfree, dtype=np.uint64)
    got = entries_variable_elimination(spec, ys, tensors=tens)
    xs = np.zeros(len(ys), dtype=np.int64)
    for q, v in fixed.items():
        xs |= v << q
    for i, q in enumerate(free):
        xs |= ((ys.astype(np.int64) >> i) & 1) << q
    assert np.abs(got - full[xs]).max() <= 1e-15 * np.abs(full).max()
