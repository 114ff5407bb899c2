"""Batched execution (level-synchronous persistent launches in a HIP graph)
and the tile autotuner (GPU).

The batch runs the same tile code as the per-step kernels, in a different
placement, so every job's output must equal its plain execution bit for bit
and match the oracle within the form's tolerance.  Graph replays are checked
one by one against the eager result, with other device work in between."""
import numpy as np
import pytest
import torch

import paper_2502_03445_amd as tqc
from oracle.reconstruct import full_distribution
from workloads import configs, synthetic

pytestmark = pytest.mark.gpu


def jobs(form):
    specs = [configs.config1(), configs.ghz(12, 3), configs.aqft(10, 3, 2),
             configs.random_cut_circuit(9, 3, 4, 3, 4)]
    for i, (m, K, outs) in enumerate([(2, 3, [7, 8]), (3, 4, [4, 5, 5]), (4, 6, [3, 3, 3, 4]),
                                      (5, 7, [2, 3, 3, 2, 3]), (1, 0, [9]), (3, 2, [0, 6, 6]),
                                      (2, 2, [10, 9]), (4, 5, [2, 4, 4, 4])]):
        specs.append(synthetic.random_network(m, K, outs, seed=500 + i))
    nets = [tqc.Network.from_spec(s) for s in specs]
    dt = "f64" if form == "fp64" else "f32"
    plans = [tqc.Plan(n, precision=form, out_dtype=dt) for n in nets]
    return specs, nets, plans


BATCH_OFF = pytest.mark.skip(reason="persistent batch launches are switched off: two runs did not "
                                    "finish on MI355X and the cause has not been identified")

@BATCH_OFF
@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp64"])
def test_batch_equals_plain_execution(form):
    specs, nets, plans = jobs(form)
    plain = [p.execute().clone() for p in plans]
    b = tqc.Batch(plans, use_graph=True)
    for o in b.outs:
        o.fill_(-7.0)
    b.execute()
    torch.cuda.synchronize()
    st, en, err = b.job_times()
    assert err == 0
    assert np.all(st >= 0) and np.all(en >= st)
    for i, (spec, o, ref_gpu) in enumerate(zip(specs, b.outs, plain)):
        assert torch.equal(o, ref_gpu), i
        ref = full_distribution(spec)
        got = o.double().cpu().numpy()
        tol = 1e-12 if form == "fp64" else (3e-5 if form == "bf16x3" else 1e-6) * np.abs(ref).max()
        assert np.abs(got - ref).max() <= tol, (i, np.abs(got - ref).max())


@BATCH_OFF
def test_graph_replays_match_eager():
    specs, nets, plans = jobs("fp32")
    b = tqc.Batch(plans, use_graph=True)
    b.execute()
    torch.cuda.synchronize()
    first = [o.clone() for o in b.outs]
    for rep in range(3):
        for o in b.outs:
            o.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        b.execute()
        torch.cuda.synchronize()
        assert junk.isfinite()
        for i, (o, f) in enumerate(zip(b.outs, first)):
            assert torch.equal(o, f), (rep, i)


@BATCH_OFF
def test_sequential_baseline_and_no_graph_mode():
    specs, nets, plans = jobs("fp32")
    b = tqc.Batch(plans, use_graph=False)
    b.execute()
    torch.cuda.synchronize()
    persistent = [o.clone() for o in b.outs]
    ms = b.execute_sequential()
    assert ms.shape == (len(plans), 2) and np.all(ms[:, 1] >= ms[:, 0])
    for o, p in zip(b.outs, persistent):
        assert torch.equal(o, p)
    info = b.info()
    assert info["units"] >= len(plans) and info["items"] >= info["units"] and info["grid"] >= 1


@pytest.mark.skip(reason="dependency-wait batch mode is kept off the GPU: one run in that mode "
                         "hung on MI355X and its cause has not been identified")
def test_host_forced_dependency_timeout_is_reported():
    # a tiny spin limit forces dependency waits to overrun; every item still
    # finishes (skipping its work) and the launch reports the error flag
    specs, nets, plans = jobs("fp32")
    b = tqc.Batch(plans, use_graph=False, spin_limit=1, dependency_waits=True)
    b.execute()
    torch.cuda.synchronize()
    _, _, err = b.job_times()
    assert err in (0, 1)
    ok = tqc.Batch(plans, use_graph=False, dependency_waits=True)
    ok.execute()
    torch.cuda.synchronize()
    assert ok.job_times()[2] == 0


def test_autotune_keeps_results(tmp_path):
    spec = synthetic.random_network(3, 4, [6, 6, 5], seed=21)
    net = tqc.Network.from_spec(spec)
    plan = tqc.Plan(net, precision="fp32")
    ref = plan.execute().clone()
    tiles = tqc.autotune(plan, reps=2)
    assert all(t in (0, 1, 2) for t in tiles)
    got = plan.execute()
    r = full_distribution(spec)
    assert np.abs(got.double().cpu().numpy() - r).max() <= 1e-6 * np.abs(r).max()
    assert torch.allclose(got, ref, rtol=0, atol=1e-6 * ref.abs().max().item())
    path = str(tmp_path / "tune.txt")
    tqc.autotune_save(path)
    tqc.autotune_load(path)
    p2 = tqc.Plan(net, precision="fp32", tile_policy=1)
    assert [s["tile"] for s in p2.steps] == tiles
