"""Heavy state selection (Sec. IV, Alg. 1) on the GPU against the oracle.

Column norms are float64 sums in a different order on each side, so the
selected subsets are compared exactly where the norms are apart and checked
for validity (every kept state at least as heavy, by the oracle's norms, as
every state left out, up to rounding) where near-ties could order them
differently.  The restricted network is contracted by the ordinary path and
compared entry by entry with the oracle at the retained product states."""
import numpy as np
import pytest
import torch

import paper_2502_03445_amd as tqc
from oracle import hss
from oracle.reconstruct import entries_bruteforce, entries_variable_elimination
from workloads import batch, configs

pytestmark = pytest.mark.gpu


def cases():
    return [(configs.ghz(12, 3), 8), (configs.w_state(12, 3), 120), (configs.aqft(10, 3, 2), 50),
            (configs.random_cut_circuit(10, 3, 4, 3, 0), 1), (configs.random_cut_circuit(10, 3, 4, 3, 1), 7),
            (configs.random_cut_circuit(10, 3, 4, 3, 2), 64), (configs.random_cut_circuit(10, 3, 4, 3, 3), 300),
            (batch.job(58), 256)]


def valid_selection(sub_gpu, norms_ref, s_max, rtol=1e-12):
    sizes = [len(s) for s in sub_gpu]
    total = int(np.prod(sizes))
    full = int(np.prod([len(n) for n in norms_ref]))
    if total < min(s_max, full):
        return False
    kept, left = [], []
    for s, nv in zip(sub_gpu, norms_ref):
        top = float(np.max(nv))
        if not any(abs(nv[i] - top) <= rtol * top for i in s):
            return False
        k = [nv[i] for i in s]
        kept += sorted(k)[:-1]  # the heaviest of each subset is its start
        left += [nv[i] for i in range(len(nv)) if i not in set(s)]
    if kept and left:
        return min(kept) >= max(left) * (1 - rtol) - 1e-300
    return True


@pytest.mark.parametrize("case", range(8))
def test_selection_matches_oracle(case):
    spec, s_max = cases()[case]
    N = tqc.Network.from_spec(spec)
    sub_gpu, norms_gpu = N.hss_select(s_max)
    sub_ref, norms_ref = hss.heavy_states(spec, s_max)
    for a, b in zip(norms_gpu, norms_ref):
        assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())
    same = all(np.array_equal(a, b) for a, b in zip(sub_gpu, sub_ref))
    assert same or valid_selection(sub_gpu, norms_ref, s_max), (case, sub_gpu, sub_ref)


def gpu_index_map(subsets):
    """oracle product order (tensor 0 fastest, mixed radix) -> padded index"""
    bits = [max(0, int(len(s) - 1).bit_length()) for s in subsets]
    offs = np.cumsum([0] + bits[:-1])
    total = int(np.prod([len(s) for s in subsets]))
    c = np.arange(total, dtype=np.int64)
    g = np.zeros(total, dtype=np.int64)
    for s, o in zip(subsets, offs):
        g |= (c % len(s)) << int(o)
        c //= len(s)
    return g, int(sum(bits))


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("case", range(8))
def test_restricted_network_reconstructs_retained_states(case, form):
    spec, s_max = cases()[case]
    N = tqc.Network.from_spec(spec)
    subsets, _ = hss.heavy_states(spec, s_max)  # the oracle's subsets on both sides
    sub = N.select_states(subsets)
    plan = tqc.Plan(sub, precision=form, out_dtype="f64" if form == "fp64" else "f32")
    got = plan.execute().double().cpu().numpy()
    gidx, nbits = gpu_index_map(subsets)
    assert got.shape == (1 << nbits,)
    xs = hss.product_indices(spec, subsets)
    ref = entries_bruteforce(spec, xs) if spec.num_cuts <= 6 else entries_variable_elimination(spec, xs)
    tol = 1e-12 if form == "fp64" else 1e-6 * max(np.abs(ref).max(), 1e-300)
    assert np.abs(got[gidx] - ref).max() <= tol
    pad = np.ones(got.shape, dtype=bool)
    pad[gidx] = False
    assert np.all(got[pad] == 0.0)
    assert abs(got.sum() - ref.sum()) <= max(tol * len(ref), 1e-12)


def test_ghz32_heavy_states_hold_all_probability():
    # full-size closed form: GHZ-32 cut into 4, 2^4 retained states hold P = 1
    spec = configs.ghz(32, 4)
    N = tqc.Network.from_spec(spec)
    subsets, _ = N.hss_select(16)
    assert [len(s) for s in subsets] == [2, 2, 2, 2]
    for s, t in zip(subsets, spec.tensors):
        assert list(s) == [0, (1 << len(t.outputs)) - 1]
    sub = N.select_states(subsets)
    got = tqc.Plan(sub, precision="fp32").execute().double().cpu().numpy()
    assert got.shape == (16,)
    assert abs(got[0] - 0.5) <= 1e-6 and abs(got[15] - 0.5) <= 1e-6
    assert abs(got.sum() - 1.0) <= 1e-6


def test_select_states_rejects_bad_subsets():
    spec = configs.ghz(12, 3)
    N = tqc.Network.from_spec(spec)
    with pytest.raises(tqc.TqcError):
        N.select_states([np.array([3, 1]), np.array([0]), np.array([0])])   # not ascending
    with pytest.raises(tqc.TqcError):
        N.select_states([np.array([0, 99]), np.array([0]), np.array([0])])  # out of range
    with pytest.raises(tqc.TqcError):
        N.select_states([np.array([], dtype=np.int32), np.array([0]), np.array([0])])
