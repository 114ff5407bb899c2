"""Pins of the heavy-state-selection oracle (Alg. 1, Eqs. (9)-(13)) against
closed forms of GHZ, W and AQFT circuits and against properties the
algorithm's output must have on any input."""
import numpy as np

from oracle import hss
from oracle.reconstruct import entries_bruteforce, full_distribution
from workloads import configs


def reconstruct_selected(net, subsets):
    xs = hss.product_indices(net, subsets)
    return xs, entries_bruteforce(net, xs)


def test_ghz_two_heavy_states_per_piece_capture_everything():
    # GHZ: P(0^n) = P(1^n) = 1/2; every piece's only non-zero columns are its
    # all-0 and all-1 states, so 2^m retained product states hold P = 1
    net = configs.ghz(12, 3)
    subsets, norms = hss.heavy_states(net, 2 ** 3)
    for (cut_ids, outs, _), s in zip([(t.cut_ids, t.outputs, None) for t in net.tensors], subsets):
        assert list(s) == [0, (1 << len(outs)) - 1]
    xs, p = reconstruct_selected(net, subsets)
    assert len(xs) == 8 and 0 in xs and (1 << 12) - 1 in xs
    assert abs(p.sum() - 1.0) <= 1e-12
    m = hss.metrics(p, full_distribution(net), net.n)
    assert abs(m["P_HSS_max"] - 1.0) <= 1e-12 and abs(m["r_P"] - 1.0) <= 1e-12


def test_w_state_all_nonzero_states_capture_everything():
    # W: P(e_i) = 1/n; a piece with o output qubits has o + 1 non-zero
    # columns (all-0 and o one-hot), so prod (o_j + 1) retained states hold
    # every e_i
    net = configs.w_state(12, 3)
    s_max = int(np.prod([len(t.outputs) + 1 for t in net.tensors]))
    subsets, norms = hss.heavy_states(net, s_max)
    for s, t in zip(subsets, net.tensors):
        o = len(t.outputs)
        assert sorted(s) == [0] + [1 << b for b in range(o)]
    xs, p = reconstruct_selected(net, subsets)
    assert abs(p.sum() - 1.0) <= 1e-12
    onehot = [1 << q for q in range(12)]
    assert all(x in xs for x in onehot)


def test_aqft_uniform_output_gives_unit_ratio():
    # AQFT on a basis state: P = 2^-n everywhere, so any |HSS| states hold
    # exactly |HSS| / 2^n: r_P = 1 and eta = 1
    net = configs.aqft(10, 3, 2)
    subsets, _ = hss.heavy_states(net, 50)
    xs, p = reconstruct_selected(net, subsets)
    m = hss.metrics(p, full_distribution(net), net.n)
    assert abs(m["r_P"] - 1.0) <= 1e-12 and abs(m["eta"] - 1.0) <= 1e-12
    assert abs(m["P_HSS"] - len(xs) / 2 ** 10) <= 1e-12


def test_selection_properties_on_random_circuits():
    for seed in range(4):
        net = configs.random_cut_circuit(10, 3, 4, 3, seed)
        for s_max in (1, 7, 64, 300):
            subsets, norms = hss.heavy_states(net, s_max)
            sizes = [len(s) for s in subsets]
            total = int(np.prod(sizes))
            full = int(np.prod([len(nv) for nv in norms]))
            # stops at the first product >= s_max (or when every state is in)
            assert total >= min(s_max, full)
            # each subset holds its heaviest state
            for s, nv in zip(subsets, norms):
                assert int(np.argmax(nv)) in s
            # the other retained states are a prefix of the global descending
            # order: none is lighter than a state left out
            kept, left = [], []
            for j, (s, nv) in enumerate(zip(subsets, norms)):
                top = int(np.argmax(nv))
                for i, v in enumerate(nv):
                    if i != top:
                        (kept if i in s else left).append(v)
            if kept and left:
                assert min(kept) >= max(left)
            # minimal: without the last state added the product was below s_max
            if total > 1 and total < full and s_max > 1:
                smallest = min(min(nv[i] for i in s if i != int(np.argmax(nv))) if len(s) > 1 else np.inf
                               for s, nv in zip(subsets, norms))
                j = [k for k, (s, nv) in enumerate(zip(subsets, norms)) if len(s) > 1 and
                     min(nv[i] for i in s if i != int(np.argmax(nv))) == smallest][-1]
                assert total // sizes[j] * (sizes[j] - 1) < s_max


def test_product_indices_cover_each_combination_once():
    net = configs.random_cut_circuit(9, 3, 3, 2, 5)
    subsets, _ = hss.heavy_states(net, 40)
    xs = hss.product_indices(net, subsets)
    assert len(np.unique(xs)) == len(xs) == int(np.prod([len(s) for s in subsets]))
    # reading each tensor's output bits back gives a member of its subset
    for t, s in zip(net.tensors, subsets):
        col = np.zeros(len(xs), dtype=np.int64)
        for b, q in enumerate(t.outputs):
            col |= ((xs >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << b
        assert np.isin(col, s).all()
