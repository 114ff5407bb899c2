"""The seeded batch of uneven reconstructions (CPU): determinism, the drawn
ranges and generation caps, and exactness of its subcircuit tensors, pinned
by reconstructing with the oracle and comparing with the uncut circuit's own
statevector probabilities (Eq. (1) holds exactly for any cut placement)."""
import numpy as np

from oracle.reconstruct import entries_variable_elimination, full_distribution
from workloads import batch
from workloads.circuit import probabilities
from workloads.cutting import cut_shapes


def test_draws_are_seeded_and_within_ranges():
    seen_k = set()
    for i in range(48):
        a = batch.draw(i)
        b = batch.draw(i)
        n, m, layout, depth, circ, sub, home, target = a
        assert (n, m, layout, depth) == b[:4] and len(circ.gates) == len(b[4].gates)
        assert all(g1 == g2 for g1, g2 in zip(circ.gates, b[4].gates))
        assert 16 <= n <= 28 and 2 <= m <= 5 and 4 <= depth <= 8 and layout in ("line", "grid")
        cuts, shapes = cut_shapes(circ, sub, num_subs=m, idle_sub=home)
        assert 2 <= len(cuts) <= 10 and len(cuts) <= target
        assert sum(s["outputs"] for s in shapes) == n
        assert all(s["width"] == s["outputs"] + s["u"] for s in shapes)
        assert sum(4 ** s["d"] * (s["gates"] + 3 ** s["u"]) * 2 ** s["width"] for s in shapes) <= batch.SIM_CAP
        flops, largest = batch.contraction_estimate(cuts, [s["outputs"] for s in shapes])
        assert flops <= batch.FLOP_CAP and largest <= batch.INTER_CAP
        seen_k.add(len(cuts))
    assert len(seen_k) >= 5


def test_cut_shapes_match_the_cut_network():
    net = batch.job(58)
    n, m, layout, depth, circ, sub, home, target = batch.draw(58)
    cuts, shapes = cut_shapes(circ, sub, num_subs=m, idle_sub=home)
    assert cuts == net.cuts
    for s, t in zip(shapes, net.tensors):
        assert t.data.shape == (4 ** s["d"] * 3 ** s["u"], 2 ** (s["outputs"] + s["u"]))
        assert len(t.outputs) == s["outputs"]


def test_few_cut_job_reconstructs_its_circuit():
    net = batch.job(158)          # 16 qubits, 5 subcircuits, 2 cuts
    assert net.n == 16 and net.num_cuts == 2
    p = probabilities(net.meta["circuit"])
    assert np.abs(full_distribution(net) - p).max() <= 1e-14


def test_ten_cut_job_reconstructs_its_circuit():
    net = batch.job(58)           # 16 qubits, 5 subcircuits, 10 cuts
    assert net.num_cuts == 10
    p = probabilities(net.meta["circuit"])
    xs = np.random.default_rng(3).choice(1 << net.n, 256, replace=False).astype(np.uint64)
    xs = np.concatenate([xs, [np.uint64(np.argmax(p))]])
    got = entries_variable_elimination(net, xs)
    assert np.abs(got - p[xs.astype(np.int64)]).max() <= 1e-14


def test_describe_counts_every_job():
    nets = [batch.job(i) for i in (158, 285, 335)]
    d = batch.describe(nets)
    assert d["jobs"] == 3 and sum(d["n_hist"].values()) == 3 and sum(d["k_hist"].values()) == 3
    assert d["output_bytes_f32"] == sum(4 << x.n for x in nets)
