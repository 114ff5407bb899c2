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


def test_multi_options_rejected_before_any_device_work():
    """tqc_multi_create_ex checks its options before it touches a plan's
    workspace or the device: a grouping mode outside 0..2 or more than 16
    streams is INVALID_ARG (the output pointers are never read)."""
    ok = [([0], [0], "pauli", np.ones((4, 2))), ([0], [1], "pauli", np.ones((4, 2)))]
    plan = tqc.Plan(_net(2, ok, [(0, 1)]))
    L = tqc.lib()
    ph = (ctypes.c_void_p * 1)(plan.handle.value)
    oh = (ctypes.c_void_p * 1)(0x1000)  # never dereferenced
    h = ctypes.c_void_p()
    for grouped, streams in ((3, 4), (-1, 4), (1, 17)):
        opt = tqc.MultiOptions(1, streams, 0, grouped, 1)
        st = L.tqc_multi_create_ex(1, ph, oh, None, ctypes.byref(opt), None, ctypes.byref(h))
        assert st == 1 and not h.value, (grouped, streams, st)


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


# ----------------------------------------------------------- plan blobs
def _plan_fields(P):
    st = dict(P.stats)
    st.pop("plan_seconds")
    return st, P.steps, P.sliced


@pytest.mark.parametrize("opts", [dict(precision="fp32"),
                                  dict(precision="fp64", out_dtype="f64", sliced=[1, 4]),
                                  dict(precision="bf16x6", fixed={0: 1, 5: 0, 9: 1}),
                                  dict(precision="fp16x3", order=[(3, 1), (4, 0), (5, 2)])])
def test_plan_blob_round_trip(opts):
    spec = synthetic.random_network(4, 7, [3, 3, 2, 4], seed=91)
    net = tqc.Network.from_spec(spec)
    P = tqc.Plan(net, **opts)
    blob = P.serialize()
    assert blob[:8] == b"TQCPLAN1"
    Q = tqc.Plan.deserialize(net, blob)
    assert _plan_fields(Q) == _plan_fields(P)
    assert Q.out_dtype == P.out_dtype
    assert Q.serialize() == blob
    # same structure, other values: the plan applies
    spec2 = synthetic.random_network(4, 7, [3, 3, 2, 4], seed=91)
    for t in spec2.tensors:
        t.data[...] = t.data[::-1]
    R = tqc.Plan.deserialize(tqc.Network.from_spec(spec2), blob)
    assert R.steps == P.steps


def test_plan_blob_budget_sliced_plan_keeps_slicing_order():
    spec = synthetic.random_network(5, 14, [2, 2, 2, 2, 2], seed=9)
    net = tqc.Network.from_spec(spec)
    free = tqc.Plan(net, precision="fp64", out_dtype="f64")
    P = tqc.Plan(net, precision="fp64", out_dtype="f64", mem_budget=free.stats["workspace_bytes"] // 3)
    assert len(P.sliced) >= 1
    Q = tqc.Plan.deserialize(net, P.serialize())
    assert Q.sliced == P.sliced and Q.steps == P.steps


def test_plan_blob_errors():
    spec = synthetic.random_network(3, 4, [3, 3, 3], seed=5)
    net = tqc.Network.from_spec(spec)
    P = tqc.Plan(net)
    blob = P.serialize()
    L = tqc.lib()
    # too small a buffer: SHAPE, and the size is reported
    n = ctypes.c_uint64(len(blob) - 1)
    buf = ctypes.create_string_buffer(len(blob))
    assert L.tqc_plan_serialize(P.handle, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)) == 3
    for bad in (blob[:-1], blob[:20], b"X" + blob[1:], blob[:40] + bytes([blob[40] ^ 1]) + blob[41:]):
        with pytest.raises(tqc.TqcError) as e:
            tqc.Plan.deserialize(net, bad)
        assert e.value.status == 1
    # another structure: TOPOLOGY
    other = tqc.Network.from_spec(synthetic.random_network(3, 4, [3, 3, 3], seed=6))
    with pytest.raises(tqc.TqcError) as e:
        tqc.Plan.deserialize(other, blob)
    assert e.value.status == 2


def test_plan_workspace_query_covers_the_plan():
    spec = synthetic.random_network(4, 7, [3, 3, 2, 4], seed=91)
    net = tqc.Network.from_spec(spec)
    for opts in (dict(), dict(precision="fp64", out_dtype="f64", sliced=[2]), dict(sliced=[0, 3])):
        P = tqc.Plan(net, **opts)
        need = P.workspace_bytes
        assert need % 256 == 0
        # at least the planner's workspace and, for a sliced float32 plan,
        # the float64 accumulator of the slice sum (both in the stats figure)
        assert need >= P.stats["workspace_bytes"]
    L = tqc.lib()
    n = ctypes.c_uint64(0)
    assert L.tqc_topk_workspace_bytes(1 << 20, 100, ctypes.byref(n)) == 0 and n.value > 0
    assert L.tqc_topk_workspace_bytes(10, 11, ctypes.byref(n)) == 1
    assert L.tqc_marginal_workspace_bytes(20, 3, ctypes.byref(n)) == 0 and n.value > 0
    assert L.tqc_marginal_workspace_bytes(20, 25, ctypes.byref(n)) == 1


# ----------------------------------------- batch launch emulated on the host
def _batch_jobs(form):
    from workloads import configs
    specs = [configs.config1(), configs.ghz(12, 3), configs.aqft(10, 3, 2),
             configs.random_cut_circuit(9, 3, 4, 3, 4)]
    for i, (m, K, outs) in enumerate([(2, 3, [7, 8]), (3, 4, [4, 5, 5]), (4, 6, [3, 3, 3, 4]),
                                      (5, 7, [2, 3, 3, 2, 3]), (1, 0, [9]), (3, 2, [0, 6, 6]),
                                      (2, 2, [10, 9]), (4, 5, [2, 4, 4, 4])]):
        specs.append(synthetic.random_network(m, K, outs, seed=500 + i))
    dt = "f64" if form == "fp64" else "f32"
    return [tqc.Plan(tqc.Network.from_spec(s), precision=form, out_dtype=dt) for s in specs]


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16x6", "fp64"])
def test_batch_launch_emulation_finds_every_access_in_bounds(form):
    """The twelve jobs of the GPU batch tests: every pre-pass and item access
    inside its buffer, loops bounded, levels and dependencies ordered."""
    plans = _batch_jobs(form)
    assert tqc.batch_validate(plans) == ""


def test_batch_launch_emulation_catches_an_undersized_output():
    plans = _batch_jobs("fp32")
    need = [p.out_entries * 4 for p in plans]
    need[3] -= 4
    rep = tqc.batch_validate(plans, need)
    assert "job 3 output" in rep, rep
