"""Host-side tests of the C-ABI (no GPU): the library loads and exports every
symbol declared in include/tqc.h, network validation errors, planner
invariants and the Sec. III-C worked example through the library."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2502_03445_amd as tqc
from oracle import plancost
from workloads import configs, qaoa, synthetic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(tqc_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = tqc.lib()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert L.tqc_version() >= 100


def _net(n, tensors, cuts):
    return tqc.Network(n, tensors, cuts)


def test_validation_errors():
    ok = [([0], [0], "pauli", np.ones((4, 2))), ([0], [1], "pauli", np.ones((4, 2)))]
    _net(2, ok, [(0, 1)])
    with pytest.raises(tqc.TqcError) as e:  # cut to itself
        _net(2, ok, [(0, 0)])
    assert e.value.status == 2
    with pytest.raises(tqc.TqcError) as e:  # qubit owned twice
        _net(2, [([0], [0], "pauli", np.ones((4, 2))), ([0], [0], "pauli", np.ones((4, 2)))], [(0, 1)])
    assert e.value.status == 2
    with pytest.raises(tqc.TqcError) as e:  # qubit never owned
        _net(3, ok, [(0, 1)])
    assert e.value.status == 2
    with pytest.raises(tqc.TqcError) as e:  # cut listed in only one tensor
        _net(2, [([0], [0], "pauli", np.ones((4, 2))), ([], [1], "pauli", np.ones((1, 2)))], [(0, 1)])
    assert e.value.status == 2
    bad = np.ones((4, 2))
    bad[1, 1] = np.nan
    with pytest.raises(tqc.TqcError) as e:  # non-finite
        _net(2, [([0], [0], "pauli", bad), ([0], [1], "pauli", np.ones((4, 2)))], [(0, 1)])
    assert e.value.status == 1


def test_worked_example_through_library():
    cut_lists = [[0], [0, 1, 2], [1, 3], [2, 3]]
    cuts = [(0, 1), (1, 2), (1, 3), (2, 3)]
    W = _net(0, [(cl, [], "pauli", np.ones((4 ** len(cl), 1))) for cl in cut_lists], cuts)
    P = tqc.Plan(W, order=[(0, 1), (4, 2), (5, 3)])
    assert P.stats["mults_per_state"] == 144
    assert P.stats["k_max_cuts"] == 3
    ref = plancost.sequence_cost([set(c) for c in cut_lists], [0] * 4, [(0, 1), (4, 2), (5, 3)],
                                 count_outputs=False)
    assert sum(ref) == 144
    # the planner's own choice is never worse than the printed order
    assert tqc.Plan(W).stats["mults_per_state"] <= 144


def test_plan_flops_match_independent_count():
    net = qaoa.qaoa_network()
    N = tqc.Network.from_spec(net)
    P = tqc.Plan(N)
    order = [(s["lhs"], s["rhs"]) for s in P.steps]
    cuts = [set(t.cut_ids) for t in net.tensors]
    outs = [len(t.outputs) for t in net.tensors]
    ref = plancost.sequence_cost(cuts, outs, order, count_outputs=True)
    assert P.stats["flops"] == pytest.approx(2 * sum(ref))
    assert P.stats["out_entries"] == 1 << 32
    # Eq. (4) bound: every step costs at most 4^Kmax per output state
    assert P.stats["mults_per_state"] <= (N.m - 1) * 4 ** P.stats["k_max_cuts"]


def test_bad_order_rejected():
    net = configs.config1()
    N = tqc.Network.from_spec(net)
    with pytest.raises(tqc.TqcError):
        tqc.Plan(N, order=[(0, 0)])


def test_fixed_qubits_and_explicit_slicing():
    spec = synthetic.random_network(4, 6, [3, 3, 2, 2], seed=5)
    N = tqc.Network.from_spec(spec)
    P = tqc.Plan(N, fixed={0: 1, 5: 0}, sliced=[1, 3])
    assert P.stats["out_qubits"] == spec.n - 2
    assert P.stats["num_slices"] == 16
    assert sorted(P.sliced) == [1, 3]
    with pytest.raises(tqc.TqcError):
        tqc.Plan(N, fixed={0: 2})


def test_memory_budget_slicing():
    # cut-heavy network with a small output: intermediates dominate memory
    spec = synthetic.random_network(5, 12, [2, 2, 2, 2, 2], seed=9)
    N = tqc.Network.from_spec(spec)
    free = tqc.Plan(N, out_dtype="f64")
    budget = free.stats["workspace_bytes"] // 3
    P = tqc.Plan(N, out_dtype="f64", mem_budget=budget)
    assert P.stats["num_sliced"] >= 1
    assert P.stats["workspace_bytes"] <= budget
    with pytest.raises(tqc.TqcError) as e:
        tqc.Plan(N, out_dtype="f64", mem_budget=64)
    assert e.value.status == 5
