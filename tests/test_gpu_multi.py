"""Many independent reconstructions as one HIP graph (GPU).

Each job runs the same launches as its plan's own execute, only on one of a
few worker streams and, with a graph, replayed from one capture; so every
output must equal the plan's plain execution bit for bit, and match the
oracle within the form's tolerance.  Graph replays are checked one by one
against the eager result, with unrelated device work and host waits between
them."""
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
                                      (2, 2, [10, 9]), (4, 5, [2, 4, 4, 4]), (2, 4, [8, 9])]):
        specs.append(synthetic.random_network(m, K, outs, seed=700 + i))
    nets = [tqc.Network.from_spec(s) for s in specs]
    dt = "f64" if form == "fp64" else "f32"
    plans = [tqc.Plan(n, precision=form, out_dtype=dt) for n in nets]
    return specs, nets, plans


def tol(form, ref):
    if form == "fp64":
        return 1e-12
    return (3e-5 if form == "bf16x3" else 1e-6) * np.abs(ref).max()


@pytest.mark.parametrize("form,use_graph,streams", [("fp32", True, 4), ("bf16x3", True, 3),
                                                    ("fp64", True, 4), ("fp32", False, 4),
                                                    ("bf16x6", False, 1), ("fp16x3", True, 4)])
def test_multi_equals_plain_execution(form, use_graph, streams):
    specs, nets, plans = jobs(form)
    plain = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=use_graph, streams=streams)
    for o in mj.outs:
        o.fill_(-7.0)
    mj.execute()
    torch.cuda.synchronize()
    for i, (spec, o, ref_gpu) in enumerate(zip(specs, mj.outs, plain)):
        assert torch.equal(o, ref_gpu), i
        ref = full_distribution(spec)
        got = o.double().cpu().numpy()
        assert np.abs(got - ref).max() <= tol(form, ref), (i, np.abs(got - ref).max())


def test_graph_replays_match_eager():
    specs, nets, plans = jobs("fp32")
    eager = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=True, streams=4, timed=True)
    for rep in range(4):
        for o in mj.outs:
            o.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        mj.execute()
        torch.cuda.synchronize()
        assert junk.isfinite()
        for i, (o, e) in enumerate(zip(mj.outs, eager)):
            assert torch.equal(o, e), (rep, i)
        st, en = mj.job_times()
        assert np.all(st >= 0) and np.all(en >= st), rep


def test_sequential_jobs_do_not_overlap():
    specs, nets, plans = jobs("fp32")
    mj = tqc.Multi(plans, use_graph=False, streams=1, timed=True)
    mj.execute()
    st, en = mj.job_times()
    order = np.argsort(st, kind="stable")
    assert np.all(en >= st)
    # one stream: each job starts after the previous one ended
    assert np.all(st[order][1:] >= en[order][:-1])
    # launched largest predicted first
    pred = np.array([p.stats["predicted_seconds"] for p in plans])
    assert np.all(np.diff(pred[order]) <= 1e-15)


def test_multi_rejects_bad_jobs():
    specs, nets, plans = jobs("fp32")
    with pytest.raises(tqc.TqcError):
        tqc.Multi([plans[0], plans[0]], outs=[plans[0].output_tensor(), plans[0].output_tensor()])
    small = torch.empty(4, device="cuda")
    with pytest.raises(tqc.TqcError):
        tqc.Multi([plans[0]], outs=[small])
    with pytest.raises(tqc.TqcError):
        tqc.Multi(plans[:2], streams=17)
    opt = tqc.MultiOptions(1, 4, 0, 3, 1)  # grouped outside 0..2
    ph = (tqc.ctypes.c_void_p * 2)(*[p.handle.value for p in plans[:2]])
    keep = [p.output_tensor() for p in plans[:2]]
    oh = (tqc.ctypes.c_void_p * 2)(*[o.data_ptr() for o in keep])
    h = tqc.ctypes.c_void_p()
    assert tqc.lib().tqc_multi_create_ex(2, ph, oh, None, tqc.ctypes.byref(opt), None, tqc.ctypes.byref(h)) != 0
    untimed = tqc.Multi(plans[:2])
    untimed.execute()
    with pytest.raises(tqc.TqcError):
        untimed.job_times()
    timed = tqc.Multi(plans[:2], timed=True)
    with pytest.raises(tqc.TqcError):
        timed.job_times()  # nothing ran yet


@pytest.mark.parametrize("form,rtol", [("fp32", 1e-6), ("bf16x6", 1e-6), ("bf16x3", 3e-5), ("fp16x3", 1e-6)])
def test_generated_batch_jobs_match_oracle(form, rtol):
    from oracle.reconstruct import entries_variable_elimination
    from workloads import batch
    specs = [batch.job(i) for i in (158, 285, 335, 58, 170, 428)]  # 16-17 qubits, 2..10 cuts
    nets = [tqc.Network.from_spec(s) for s in specs]
    plans = [tqc.Plan(n, precision=form) for n in nets]
    plain = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=True, streams=4)
    mj.execute()
    mj.execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for i, (spec, o, ref_gpu) in enumerate(zip(specs, mj.outs, plain)):
        assert torch.equal(o, ref_gpu), i
        got = o.double().cpu().numpy()
        xs = rng.choice(1 << spec.n, 512, replace=False).astype(np.uint64)
        xs = np.unique(np.concatenate([xs, np.argsort(got)[-8:].astype(np.uint64)]))
        ref = entries_variable_elimination(spec, xs)
        bound = rtol * np.abs(ref).max()
        assert np.abs(got[xs.astype(np.int64)] - ref).max() <= bound, (i, spec.num_cuts)
        assert abs(got.sum() - 1.0) <= 1e-4


# ------------------------------------------------------------ grouped mode
@pytest.mark.parametrize("form,use_graph,waves", [("fp32", True, 1), ("fp32", False, 3), ("bf16x3", True, 2),
                                                  ("bf16x6", True, 1), ("fp16x3", False, 2), ("fp64", True, 4)])
def test_grouped_equals_plain_execution(form, use_graph, waves):
    """Every kind of work of all jobs in shared launches (transform passes,
    scales, packs, steps by depth, final steps on the persistent kernel in one
    launch per (form, K)); every output still equals the plan's own
    execution bit for bit, also over graph replays."""
    specs, nets, plans = jobs(form)
    plain = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=use_graph, timed=True, grouped=True, waves=waves)
    nl, nb, nr = mj.info()
    assert 0 < nl < 4 * len(plans), nl
    if form != "fp64":
        assert nb >= 3 and 1 <= nr <= nb, (nb, nr)
    for rep in range(3):
        for o in mj.outs:
            o.fill_(-7.0)
        mj.execute()
        torch.cuda.synchronize()
        for i, (o, ref_gpu) in enumerate(zip(mj.outs, plain)):
            assert torch.equal(o, ref_gpu), (rep, i)
        st, en = mj.job_times()
        assert np.all(st == 0) and np.all(en >= st), rep
    for spec, o in zip(specs, mj.outs):
        ref = full_distribution(spec)
        assert np.abs(o.double().cpu().numpy() - ref).max() <= tol(form, ref)


@pytest.mark.parametrize("form,use_graph,waves,streams", [("fp32", True, 1, 4), ("fp32", False, 3, 2),
                                                          ("bf16x3", True, 2, 8), ("bf16x6", True, 4, 3),
                                                          ("fp16x3", True, 2, 4), ("fp64", False, 1, 1)])
def test_grouped_heads_equal_plain_execution(form, use_graph, waves, streams):
    """Grouped heads: the transforms, scales and packs of each wave's jobs in
    shared launches, then every job's own pairwise steps and final step on a
    worker stream; outputs equal the plan's own execution bit for bit, over
    graph replays with unrelated eager work between them."""
    specs, nets, plans = jobs(form)
    plain = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=use_graph, streams=streams, timed=True, grouped="heads", waves=waves)
    nl, nb, nr = mj.info()
    assert 0 < nl <= 8 * waves and nb == 0 and nr == 0, (nl, nb, nr)
    for rep in range(3):
        for o in mj.outs:
            o.fill_(-7.0)
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        mj.execute()
        torch.cuda.synchronize()
        assert junk.isfinite()
        for i, (o, ref_gpu) in enumerate(zip(mj.outs, plain)):
            assert torch.equal(o, ref_gpu), (rep, i)
        st, en = mj.job_times()
        assert np.all(st >= 0) and np.all(en >= st), rep
    for spec, o in zip(specs, mj.outs):
        ref = full_distribution(spec)
        assert np.abs(o.double().cpu().numpy() - ref).max() <= tol(form, ref)


def test_grouped_heads_large_jobs():
    """Twelve jobs of the batch workload with n 20..28 (multi-pass
    transforms, several depths, split-k steps among them) with grouped
    heads in three waves over eight streams: bit-identical to their own
    executions."""
    from workloads import batch
    ids = [18, 7, 1, 5, 28, 3, 22, 2, 16, 11, 19, 46]
    specs = [batch.job(i) for i in ids]
    plans = [tqc.Plan(tqc.Network.from_spec(s), precision="fp32") for s in specs]
    plain = [p.execute().clone() for p in plans]
    torch.cuda.synchronize()
    mj = tqc.Multi(plans, use_graph=True, streams=8, grouped="heads", waves=3)
    for o in mj.outs:
        o.fill_(-7.0)
    mj.execute()
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(mj.outs, plain)):
        assert torch.equal(o, r), ids[i]


def test_grouped_final_steps_of_many_shapes_and_ks():
    """Forty reconstructions of two tensors with outputs of 2^7..2^11 rows and
    columns and K = 16..256 in float32: their final steps go to one
    persistent launch per K, each output equal to its plan's own execution."""
    rng = np.random.default_rng(77)
    specs = []
    for i in range(40):
        K = int(rng.integers(2, 5))
        outs = [int(rng.integers(7, 12)), int(rng.integers(7, 12))]
        specs.append(synthetic.random_network(2, K, outs, seed=1900 + i))
    plans = [tqc.Plan(tqc.Network.from_spec(s), precision="fp32") for s in specs]
    plain = [p.execute().clone() for p in plans]
    mj = tqc.Multi(plans, use_graph=True, grouped=True)
    nl, nb, nr = mj.info()
    assert nb == 40 and nr == len({p.steps[-1]["log2_k"] for p in plans}), (nb, nr)
    mj.execute()
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(mj.outs, plain)):
        assert torch.equal(o, r), i


def test_grouped_large_jobs_against_oracle():
    """Twelve jobs of the batch workload with n 20..28 (exact subcircuit
    tensors; multi-pass transforms, several depths, split-k steps among
    them), grouped: bit-identical to their own executions."""
    from workloads import batch
    ids = [18, 7, 1, 5, 28, 3, 22, 2, 16, 11, 19, 46]
    specs = [batch.job(i) for i in ids]
    plans = [tqc.Plan(tqc.Network.from_spec(s), precision="fp32") for s in specs]
    plain = [p.execute().clone() for p in plans]
    torch.cuda.synchronize()
    mj = tqc.Multi(plans, use_graph=True, grouped=True, waves=3)
    mj.execute()
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(mj.outs, plain)):
        assert torch.equal(o, r), ids[i]
