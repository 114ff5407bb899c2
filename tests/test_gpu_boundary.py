"""The C-ABI boundary on the GPU: plan blobs execute bit-identically,
caller-owned (torch) workspaces give the same results as library-owned
buffers and allocate nothing on the execute path, and the scans' scratch is
never shared between streams (two top-k / marginal calls in flight at once
on two streams, each checked against the oracle)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2502_03445_amd as tqc
from oracle import outputs as oout
from oracle.reconstruct import full_distribution
from workloads import configs, synthetic

pytestmark = pytest.mark.gpu

CASES = [dict(precision="fp32"),
         dict(precision="fp64", out_dtype="f64"),
         dict(precision="fp32", sliced=[1, 4]),               # float64 slice sum into float32
         dict(precision="fp64", out_dtype="f64", sliced=[2]),
         dict(precision="bf16x6", fixed={0: 1, 5: 0, 9: 1}),
         dict(precision="fp16x3"),
         dict(precision="bf16x3", order=[(3, 1), (4, 0), (5, 2)])]


def _spec():
    return synthetic.random_network(4, 7, [4, 4, 3, 5], seed=91)


@pytest.mark.parametrize("opts", CASES)
def test_blob_round_trip_executes_bit_identically(opts):
    net = tqc.Network.from_spec(_spec())
    P = tqc.Plan(net, **opts)
    Q = tqc.Plan.deserialize(net, P.serialize())
    a = P.execute().clone()
    b = Q.execute()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_blob_keeps_autotuned_tiles():
    net = tqc.Network.from_spec(synthetic.random_network(3, 4, [6, 6, 5], seed=21))
    P = tqc.Plan(net, precision="fp32")
    tqc.autotune(P, reps=1)
    tiles = [s["tile"] for s in P.steps]
    Q = tqc.Plan.deserialize(net, P.serialize())
    assert [s["tile"] for s in Q.steps] == tiles
    assert torch.equal(P.execute().clone(), Q.execute())


@pytest.mark.parametrize("opts", CASES)
def test_torch_workspace_equals_library_buffers(opts):
    net = tqc.Network.from_spec(_spec())
    lib_plan = tqc.Plan(net, workspace="library", **opts)
    ref = lib_plan.execute().clone()
    _, ri, rv, rt, _ = lib_plan.execute_summary(k=50)
    ri, rv, rt = ri.clone(), rv.clone(), rt.clone()
    P = tqc.Plan(net, workspace="torch", **opts)
    out = P.execute()
    torch.cuda.synchronize()
    assert P._ws is not None and P._ws.numel() >= P.workspace_bytes
    assert torch.equal(out, ref)
    _, i, v, t, _ = P.execute_summary(k=50)
    torch.cuda.synchronize()
    assert torch.equal(i, ri) and torch.equal(v, rv) and torch.equal(t, rt)


def test_bound_workspace_execute_allocates_no_device_memory():
    # a sliced float32 plan of 2^26 entries: library-owned buffers would add
    # a 512 MiB float64 accumulator on the first execute
    spec = synthetic.random_network(4, 6, [7, 7, 6, 6], seed=3)
    net = tqc.Network.from_spec(spec)
    P = tqc.Plan(net, precision="fp32", sliced=[0, 3])
    out = P.output_tensor()
    P.bind_workspace()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    P.execute(out)
    P.execute_summary(out, k=100)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (64 << 20), (free0 - free1)
    L = tqc.Plan(net, precision="fp32", sliced=[0, 3], workspace="library")
    ref = L.execute()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_workspace_errors():
    net = tqc.Network.from_spec(_spec())
    P = tqc.Plan(net, precision="fp32", workspace="library")
    small = torch.empty(P.workspace_bytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(tqc.TqcError) as e:
        P.bind_workspace(small)
    assert e.value.status == 3
    big = torch.empty(P.workspace_bytes + 512, dtype=torch.uint8, device="cuda")
    L = tqc.lib()
    st = L.tqc_plan_set_workspace(P.handle, ctypes.c_void_p(big.data_ptr() + 16), P.workspace_bytes,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 1
    # a failed bind leaves the plan on library buffers: it still runs
    r = full_distribution(_spec())
    got = P.execute().double().cpu().numpy()
    assert np.abs(got - r).max() <= 1e-6 * np.abs(r).max()


@pytest.mark.parametrize("form", ["library", "torch"])
def test_scans_on_two_streams_at_once(form):
    """Two different vectors, their top-k and totals enqueued back to back on
    two streams with no wait in between; with one shared scratch buffer the
    two calls would overwrite each other's counters and candidates."""
    n = 1 << 24
    g = torch.Generator(device="cuda").manual_seed(11)
    a = torch.rand(n, device="cuda", generator=g)
    b = torch.rand(n, device="cuda", generator=g) ** 3
    b[12345] = 7.0
    b[777] = 7.0                      # a tie, smaller index first
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    res = {}
    for rep in range(3):
        with torch.cuda.stream(s1):
            ia, va = tqc.topk(a, 1000, stream=s1, workspace=form)
            ta = tqc.marginal(a, 24, [3, 17], stream=s1, workspace=form)
        with torch.cuda.stream(s2):
            ib, vb = tqc.topk(b, 1000, stream=s2, workspace=form)
            tb = tqc.marginal(b, 24, [3, 17], stream=s2, workspace=form)
        torch.cuda.synchronize()
        res[rep] = [x.cpu().numpy() for x in (ia, va, ta, ib, vb, tb)]
    for vec, (ix, vx, mx) in ((a, (0, 1, 2)), (b, (3, 4, 5))):
        h = vec.double().cpu().numpy()
        oi, ov = oout.topk(h, 1000)
        om = oout.marginal(h, 24, [3, 17])
        for rep in range(3):
            r = res[rep]
            assert np.array_equal(r[ix].astype(np.int64), np.asarray(oi, dtype=np.int64)), rep
            assert np.array_equal(r[vx], np.asarray(ov, dtype=np.float64)), rep
            assert np.allclose(r[mx], om, rtol=1e-12, atol=0), rep


def test_summary_of_sliced_plans_on_two_streams():
    """The standalone scans of a sliced plan's summary, two plans on two
    streams at once (library scratch per stream)."""
    specs = [synthetic.random_network(3, 4, [5, 5, 5], seed=s) for s in (31, 32)]
    plans = [tqc.Plan(tqc.Network.from_spec(sp), precision="fp64", out_dtype="f64", sliced=[1],
                      workspace="library") for sp in specs]
    refs = [full_distribution(sp) for sp in specs]
    s = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for P, st in zip(plans, s):
        with torch.cuda.stream(st):
            outs.append(P.execute_summary(k=64, stream=st))
    torch.cuda.synchronize()
    for (o, idx, val, tot, _), r in zip(outs, refs):
        oi, ov = oout.topk(o.cpu().numpy(), 64)
        assert np.array_equal(idx.cpu().numpy(), np.asarray(oi, dtype=np.int64))
        assert np.abs(o.cpu().numpy() - r).max() <= 1e-12
        assert abs(tot.item() - r.sum()) <= 1e-12
