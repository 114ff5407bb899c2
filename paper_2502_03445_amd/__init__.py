"""Python binding of libtqc (HIP, MI355X): reconstruction of cut quantum
circuits by tensor-network contraction.

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory and streams; torch is imported
before the library is loaded so that both share one HIP runtime.  There is
no CPU fallback: if ``libtqc.so`` is missing, loading fails.

    net  = Network(n, tensors=[(cut_ids, outputs, basis, data), ...], cuts=[(up, down), ...])
    plan = Plan(net, precision="fp32")
    out  = plan.execute()                # torch tensor on the current device
    idx, val = topk(out, k)
    tot  = marginal(out, plan.out_qubits, [])
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

__all__ = ["lib", "Network", "Plan", "Batch", "CostModel", "step_features", "topk", "marginal", "autotune", "autotune_save",
           "autotune_load", "TqcError", "PRECISIONS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtqc.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "fp16x3": 4}
DTYPES = {"f64": 0, "f32": 1}
BASES = {"raw": 0, "pauli": 1}
COST = {"flopbyte": 0, "mlp": 1, "measured": 2}

_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class TensorDesc(ctypes.Structure):
    _fields_ = [("num_cuts", ctypes.c_int32), ("cut_ids", _i32p),
                ("num_outputs", ctypes.c_int32), ("output_qubits", _i32p),
                ("basis", ctypes.c_int), ("data", _dp)]


class Cut(ctypes.Structure):
    _fields_ = [("upstream", ctypes.c_int32), ("downstream", ctypes.c_int32)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("out_dtype", ctypes.c_int),
                ("mem_budget_bytes", ctypes.c_uint64),
                ("num_fixed", ctypes.c_int32), ("fixed_qubits", _i32p), ("fixed_values", _i32p),
                ("num_order_steps", ctypes.c_int32), ("order", _i32p),
                ("num_sliced", ctypes.c_int32), ("sliced_cuts", _i32p),
                ("cost_kind", ctypes.c_int), ("cost_model", ctypes.c_void_p),
                ("num_candidates", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("tile_policy", ctypes.c_int32), ("num_measured", ctypes.c_int32),
                ("max_rel_error", ctypes.c_double)]


class PlanStats(ctypes.Structure):
    _fields_ = [("num_steps", ctypes.c_int32), ("num_sliced", ctypes.c_int32),
                ("k_max_cuts", ctypes.c_int32), ("out_qubits", ctypes.c_int32),
                ("num_slices", ctypes.c_uint64), ("out_entries", ctypes.c_uint64),
                ("flops", ctypes.c_double), ("mults_per_state", ctypes.c_double),
                ("bytes", ctypes.c_double), ("predicted_seconds", ctypes.c_double),
                ("workspace_bytes", ctypes.c_uint64), ("plan_seconds", ctypes.c_double),
                ("precision", ctypes.c_int32), ("out_dtype", ctypes.c_int32),
                ("num_measured", ctypes.c_int32), ("measured_seconds", ctypes.c_double),
                ("fallback_measured_seconds", ctypes.c_double), ("checked_rel_error", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("lhs", ctypes.c_int32), ("rhs", ctypes.c_int32), ("result", ctypes.c_int32),
                ("log2_m", ctypes.c_int32), ("log2_n", ctypes.c_int32), ("log2_k", ctypes.c_int32),
                ("shared_cuts", ctypes.c_int32), ("open_cuts", ctypes.c_int32),
                ("slice_dependent", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("dependency_waits", ctypes.c_int32), ("spin_limit", ctypes.c_uint64)]


class MultiOptions(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("num_streams", ctypes.c_int32), ("timed", ctypes.c_int32),
                ("grouped", ctypes.c_int32), ("waves", ctypes.c_int32)]


class TrainOptions(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class TqcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None


def _declare(L):
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32
    sigs = {
        "tqc_network_create": [i32, i32, ctypes.POINTER(TensorDesc), i32, ctypes.POINTER(Cut),
                               ctypes.POINTER(vp)],
        "tqc_network_upload": [vp],
        "tqc_plan_create": [vp, ctypes.POINTER(PlanOptions), ctypes.POINTER(vp)],
        "tqc_plan_get_stats": [vp, ctypes.POINTER(PlanStats)],
        "tqc_plan_get_step": [vp, i32, ctypes.POINTER(StepInfo)],
        "tqc_plan_get_sliced": [vp, _i32p],
        "tqc_execute": [vp, vp, u64, vp],
        "tqc_execute_slices": [vp, vp, u64, u64, u64, i32, vp],
        "tqc_execute_profiled": [vp, vp, u64, vp, _dp, i32],
        "tqc_execute_summary": [vp, vp, u64, i32, vp, vp, vp, _dp, i32, vp],
        "tqc_network_pauli_tensor": [vp, i32, vp, u64, vp],
        "tqc_topk": [vp, ctypes.c_int, u64, i32, vp, vp, vp],
        "tqc_marginal": [vp, ctypes.c_int, i32, i32, _i32p, vp, vp],
        "tqc_batch_create": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(u64),
                             ctypes.POINTER(BatchOptions), vp, ctypes.POINTER(vp)],
        "tqc_batch_execute": [vp, vp],
        "tqc_batch_execute_sequential": [vp, vp, _dp],
        "tqc_batch_job_times": [vp, _dp, _dp, ctypes.POINTER(ctypes.c_uint32)],
        "tqc_batch_info": [vp, ctypes.POINTER(u64), _i32p, _i32p],
        "tqc_multi_create": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(u64), i32, i32,
                             i32, vp, ctypes.POINTER(vp)],
        "tqc_multi_execute": [vp, vp],
        "tqc_multi_create_ex": [i32, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(u64),
                                ctypes.POINTER(MultiOptions), vp, ctypes.POINTER(vp)],
        "tqc_multi_info": [vp, _i32p, _i32p, _i32p],
        "tqc_hss_select": [vp, u64, _i32p, _i32p, u64, _dp, u64, vp],
        "tqc_find_cuts": [i32, i32, _i32p, i32, i32, i32, ctypes.c_double, _i32p, _i32p],
        "tqc_network_select_states": [vp, _i32p, _i32p, vp, ctypes.POINTER(vp)],
        "tqc_multi_job_times": [vp, _dp, _dp],
        "tqc_plan_autotune": [vp, vp, u64, i32, vp],
        "tqc_autotune_save": [ctypes.c_char_p],
        "tqc_autotune_load": [ctypes.c_char_p],
        "tqc_costmodel_create": [u64, ctypes.POINTER(vp)],
        "tqc_costmodel_get_params": [vp, ctypes.POINTER(ctypes.c_float), i32],
        "tqc_costmodel_set_params": [vp, ctypes.POINTER(ctypes.c_float), i32],
        "tqc_costmodel_forward": [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_float), vp],
        "tqc_costmodel_gradients": [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                    ctypes.c_int64, ctypes.POINTER(ctypes.c_float), vp],
        "tqc_costmodel_train": [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                ctypes.c_int64, ctypes.POINTER(TrainOptions),
                                ctypes.POINTER(ctypes.c_float), vp],
        "tqc_costmodel_predict": [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int64, _dp, vp],
        "tqc_costmodel_save": [vp, ctypes.c_char_p],
        "tqc_costmodel_load": [ctypes.c_char_p, ctypes.POINTER(vp)],
        "tqc_plan_step_features": [vp, ctypes.POINTER(ctypes.c_float), i32],
        "tqc_batch_validate": [i32, ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.c_char_p, u64],
        "tqc_plan_serialize": [vp, vp, ctypes.POINTER(u64)],
        "tqc_plan_deserialize": [vp, vp, u64, ctypes.POINTER(vp)],
        "tqc_plan_workspace_bytes": [vp, ctypes.POINTER(u64)],
        "tqc_plan_set_workspace": [vp, vp, u64, vp],
        "tqc_topk_workspace_bytes": [u64, i32, ctypes.POINTER(u64)],
        "tqc_topk_ws": [vp, ctypes.c_int, u64, i32, vp, vp, vp, u64, vp],
        "tqc_marginal_workspace_bytes": [i32, i32, ctypes.POINTER(u64)],
        "tqc_marginal_ws": [vp, ctypes.c_int, i32, i32, _i32p, vp, vp, u64, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.tqc_costmodel_num_params.restype = ctypes.c_int32
    L.tqc_costmodel_num_features.restype = ctypes.c_int32
    for name in ("tqc_network_destroy", "tqc_plan_destroy", "tqc_batch_destroy",
                 "tqc_multi_destroy", "tqc_costmodel_destroy"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = None
    L.tqc_plan_options_default.argtypes = [ctypes.POINTER(PlanOptions)]
    L.tqc_plan_options_default.restype = None
    L.tqc_status_string.argtypes = [ctypes.c_int]
    L.tqc_status_string.restype = ctypes.c_char_p
    L.tqc_last_error.argtypes = []
    L.tqc_last_error.restype = ctypes.c_char_p
    L.tqc_version.restype = ctypes.c_int32


def lib():
    """Load libtqc.so (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2502_03445_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _LIB = L
    return _LIB


def _check(st):
    if st != 0:
        L = lib()
        raise TqcError(st, f"{L.tqc_status_string(st).decode()}: {L.tqc_last_error().decode()}")


def _i32arr(vals):
    a = (ctypes.c_int32 * max(1, len(vals)))(*[int(v) for v in vals])
    return a


def _stream_ptr(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Network:
    """Subcircuit tensors plus cut-edge list (host copy; device upload on demand).

    tensors: sequence of (cut_ids, output_qubits, basis, data) with basis
    "raw" or "pauli" and data a float64 2-D array in the layout of tqc.h.
    cuts: sequence of (upstream_tensor, downstream_tensor)."""

    def __init__(self, n, tensors, cuts):
        L = lib()
        self._keep = []
        descs = (TensorDesc * len(tensors))()
        for d, (cids, outs, basis, data) in zip(descs, tensors):
            arr = np.ascontiguousarray(np.asarray(data, dtype=np.float64))
            ci, oq = _i32arr(cids), _i32arr(outs)
            self._keep += [arr, ci, oq]
            d.num_cuts = len(cids)
            d.cut_ids = ctypes.cast(ci, _i32p)
            d.num_outputs = len(outs)
            d.output_qubits = ctypes.cast(oq, _i32p)
            d.basis = BASES[basis]
            d.data = arr.ctypes.data_as(_dp)
        cc = (Cut * max(1, len(cuts)))(*[Cut(int(u), int(v)) for u, v in cuts])
        h = ctypes.c_void_p()
        _check(L.tqc_network_create(int(n), len(tensors), descs, len(cuts), cc, ctypes.byref(h)))
        self._keep = None
        self.handle = h
        self.n = int(n)
        self.m = len(tensors)
        self.num_cuts = len(cuts)
        self.shapes = [(len(t[0]), len(t[1])) for t in tensors]

    @classmethod
    def from_spec(cls, spec):
        """From any object with .n, .cuts and .tensors (cut_ids, outputs, basis, data)."""
        return cls(spec.n, [(t.cut_ids, t.outputs, t.basis, t.data) for t in spec.tensors], spec.cuts)

    def upload(self):
        _check(lib().tqc_network_upload(self.handle))

    def pauli_tensor(self, j, stream=None):
        c, o = self.shapes[j]
        out = torch.empty((4 ** c, 1 << o), dtype=torch.float64, device="cuda")
        _check(lib().tqc_network_pauli_tensor(self.handle, int(j), ctypes.c_void_p(out.data_ptr()),
                                              out.numel() * 8, _stream_ptr(stream)))
        return out

    def hss_select(self, s_max, stream=None):
        """Heavy state selection (Alg. 1): (subsets, norms), one int32 array of
        ascending output states and one float64 array of column norms per
        tensor."""
        widths = [1 << o for _, o in self.shapes]
        counts = (ctypes.c_int32 * self.m)()
        states = (ctypes.c_int32 * sum(widths))()
        norms = (ctypes.c_double * sum(widths))()
        _check(lib().tqc_hss_select(self.handle, int(s_max), ctypes.cast(counts, _i32p),
                                    ctypes.cast(states, _i32p), sum(widths), ctypes.cast(norms, _dp),
                                    sum(widths), _stream_ptr(stream)))
        st, nv = np.array(states[:]), np.array(norms[:])
        subsets, out_norms, a, b = [], [], 0, 0
        for j in range(self.m):
            subsets.append(st[a:a + counts[j]].astype(np.int32))
            out_norms.append(nv[b:b + widths[j]])
            a += counts[j]
            b += widths[j]
        return subsets, out_norms

    def select_states(self, subsets, stream=None):
        """The network restricted to the given output states of each tensor
        (zero-padded to powers of two); see tqc_network_select_states."""
        counts = _i32arr([len(x) for x in subsets])
        flat = _i32arr([int(v) for x in subsets for v in x])
        h = ctypes.c_void_p()
        _check(lib().tqc_network_select_states(self.handle, ctypes.cast(counts, _i32p), ctypes.cast(flat, _i32p),
                                               _stream_ptr(stream), ctypes.byref(h)))
        sub = Network.__new__(Network)
        sub._keep = None
        sub.handle = h
        sub.bits = [max(0, int(len(x) - 1).bit_length()) for x in subsets]
        sub.n = int(sum(sub.bits))
        sub.m = self.m
        sub.num_cuts = self.num_cuts
        sub.shapes = [(c, b) for (c, _), b in zip(self.shapes, sub.bits)]
        return sub

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.tqc_network_destroy(h)
            self.handle = None


def _device_bytes(nbytes, device=None):
    """A 256-byte aligned device buffer of at least nbytes from torch's
    allocator (its blocks are 512-byte aligned)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")
    assert t.data_ptr() % 256 == 0
    return t


class Plan:
    """Contraction plan: order, slicing, GEMM mapping (host-only until executed).

    workspace="torch" (default): before the first execution the plan binds
    one torch-allocated device region holding every buffer it uses
    (tqc_plan_set_workspace), so the library allocates no device memory for
    it; workspace="library": the library allocates on first use."""

    def __init__(self, net, precision="fp32", out_dtype="f32", mem_budget=0, fixed=None,
                 order=None, sliced=None, cost="flopbyte", cost_model=None, num_candidates=0,
                 seed=0, tile_policy=0, workspace="torch", num_measured=0, max_rel_error=0.0):
        if workspace not in ("torch", "library"):
            raise ValueError("workspace must be 'torch' or 'library'")
        self.workspace = workspace
        self._ws = None
        L = lib()
        o = PlanOptions()
        L.tqc_plan_options_default(ctypes.byref(o))
        o.precision = PRECISIONS[precision]
        o.out_dtype = DTYPES[out_dtype]
        o.mem_budget_bytes = int(mem_budget)
        keep = []
        if fixed:
            fq, fv = zip(*sorted(fixed.items()))
            a, b = _i32arr(fq), _i32arr(fv)
            keep += [a, b]
            o.num_fixed = len(fq)
            o.fixed_qubits = ctypes.cast(a, _i32p)
            o.fixed_values = ctypes.cast(b, _i32p)
        if order is not None:
            flat = [int(x) for pair in order for x in pair]
            a = _i32arr(flat)
            keep.append(a)
            o.num_order_steps = len(order)
            o.order = ctypes.cast(a, _i32p)
        if sliced is not None:
            a = _i32arr(sliced)
            keep.append(a)
            o.num_sliced = len(sliced)
            o.sliced_cuts = ctypes.cast(a, _i32p)
        o.cost_kind = COST[cost]
        o.cost_model = cost_model.handle if cost_model is not None else None
        o.num_candidates = int(num_candidates)
        o.seed = int(seed)
        o.tile_policy = int(tile_policy)
        o.num_measured = int(num_measured)
        o.max_rel_error = float(max_rel_error)
        h = ctypes.c_void_p()
        _check(L.tqc_plan_create(net.handle, ctypes.byref(o), ctypes.byref(h)))
        self._adopt(h, net, out_dtype)

    def _adopt(self, h, net, out_dtype):
        L = lib()
        self.handle = h
        self.net = net  # keep the network alive
        st = PlanStats()
        _check(L.tqc_plan_get_stats(h, ctypes.byref(st)))
        self.stats = {f: getattr(st, f) for f, _ in PlanStats._fields_}
        self.out_dtype = "f64" if st.out_dtype == DTYPES["f64"] else "f32"
        assert out_dtype is None or out_dtype == self.out_dtype
        self.out_qubits = st.out_qubits
        self.out_entries = st.out_entries

    def serialize(self):
        """The plan's decisions and its network's structure as bytes
        (tqc_plan_serialize)."""
        n = ctypes.c_uint64(0)
        _check(lib().tqc_plan_serialize(self.handle, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().tqc_plan_serialize(self.handle, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)))
        return bytes(buf.raw[:n.value])

    @classmethod
    def deserialize(cls, net, blob, workspace="torch"):
        """Rebuild a serialized plan on a network of the same structure."""
        blob = bytes(blob)
        buf = ctypes.create_string_buffer(blob, len(blob))
        h = ctypes.c_void_p()
        _check(lib().tqc_plan_deserialize(net.handle, ctypes.cast(buf, ctypes.c_void_p), len(blob),
                                          ctypes.byref(h)))
        p = cls.__new__(cls)
        p.workspace = workspace
        p._ws = None
        p._adopt(h, net, None)
        return p

    @property
    def workspace_bytes(self):
        n = ctypes.c_uint64(0)
        _check(lib().tqc_plan_workspace_bytes(self.handle, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, buf=None, stream=None):
        """Bind a caller-owned device region (a torch tensor; allocated here
        when None) as the plan's workspace.  Called before the first execution
        of a plan made with workspace="torch"."""
        if buf is None:
            buf = _device_bytes(self.workspace_bytes)
        _check(lib().tqc_plan_set_workspace(self.handle, ctypes.c_void_p(buf.data_ptr()),
                                            buf.numel() * buf.element_size(), _stream_ptr(stream)))
        self._ws = buf
        return buf

    def _ready(self, stream=None):
        if self.workspace == "torch" and self._ws is None:
            self.bind_workspace(stream=stream)
        if self._ws is not None and stream is not None:
            # the region is used on this stream: torch must not hand it out
            # again before that stream's work is done
            self._ws.record_stream(_torch_stream(stream))

    @property
    def steps(self):
        res = []
        for s in range(self.stats["num_steps"]):
            info = StepInfo()
            _check(lib().tqc_plan_get_step(self.handle, s, ctypes.byref(info)))
            res.append({f: getattr(info, f) for f, _ in StepInfo._fields_})
        return res

    @property
    def sliced(self):
        n = self.stats["num_sliced"]
        a = (ctypes.c_int32 * max(1, n))()
        _check(lib().tqc_plan_get_sliced(self.handle, ctypes.cast(a, _i32p)))
        return [a[i] for i in range(n)]

    def output_tensor(self, device="cuda"):
        dt = torch.float32 if self.out_dtype == "f32" else torch.float64
        return torch.empty(self.out_entries, dtype=dt, device=device)

    def execute(self, out=None, stream=None):
        if out is None:
            out = self.output_tensor()
        self._ready(stream)
        _check(lib().tqc_execute(self.handle, ctypes.c_void_p(out.data_ptr()),
                                 out.numel() * out.element_size(), _stream_ptr(stream)))
        return out

    def execute_profiled(self, out=None, stream=None):
        """Execute and return (out, phase_ms): [transform, pack, step 0.., finalize]."""
        if out is None:
            out = self.output_tensor()
        self._ready(stream)
        n = 3 + self.stats["num_steps"]
        ms = (ctypes.c_double * n)()
        _check(lib().tqc_execute_profiled(self.handle, ctypes.c_void_p(out.data_ptr()),
                                          out.numel() * out.element_size(), _stream_ptr(stream),
                                          ctypes.cast(ms, _dp), n))
        return out, [ms[i] for i in range(n)]

    def execute_summary(self, out=None, k=0, profile=False, stream=None):
        """Execute, then the k largest entries and the float64 total of the
        output.  Returns (out, idx, val, total, phase_ms or None); idx int64,
        val and total float64, on the output's device."""
        if out is None:
            out = self.output_tensor()
        dev = out.device
        self._ready(stream)
        idx = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
        val = torch.empty(max(k, 1), dtype=torch.float64, device=dev)
        tot = torch.empty(1, dtype=torch.float64, device=dev)
        n = 3 + self.stats["num_steps"]
        ms = (ctypes.c_double * n)() if profile else None
        _check(lib().tqc_execute_summary(self.handle, ctypes.c_void_p(out.data_ptr()),
                                         out.numel() * out.element_size(), int(k),
                                         ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()),
                                         ctypes.c_void_p(tot.data_ptr()),
                                         ctypes.cast(ms, _dp) if profile else None, n if profile else 0,
                                         _stream_ptr(stream)))
        return out, idx[:k], val[:k], tot, ([ms[i] for i in range(n)] if profile else None)

    def execute_slices(self, out, begin, end, accumulate=True, stream=None):
        assert out.dtype == torch.float64
        self._ready(stream)
        _check(lib().tqc_execute_slices(self.handle, ctypes.c_void_p(out.data_ptr()),
                                        out.numel() * 8, int(begin), int(end), int(bool(accumulate)),
                                        _stream_ptr(stream)))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.tqc_plan_destroy(h)
            self.handle = None


def _dtype_code(t):
    if t.dtype == torch.float32:
        return DTYPES["f32"]
    if t.dtype == torch.float64:
        return DTYPES["f64"]
    raise TypeError("probabilities must be float32 or float64")


def topk(probs, k, stream=None, workspace="torch"):
    """k largest entries (value desc, index asc): (int64 indices, float64
    values) on device.  workspace="torch" passes a torch-allocated scratch
    (tqc_topk_ws); "library" uses the library's per-stream scratch (tqc_topk)."""
    idx = torch.empty(k, dtype=torch.int64, device=probs.device)
    val = torch.empty(k, dtype=torch.float64, device=probs.device)
    L = lib()
    args = (ctypes.c_void_p(probs.data_ptr()), _dtype_code(probs), probs.numel(), int(k),
            ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(val.data_ptr()))
    if workspace == "library":
        _check(L.tqc_topk(*args, _stream_ptr(stream)))
    else:
        n = ctypes.c_uint64(0)
        _check(L.tqc_topk_workspace_bytes(probs.numel(), int(k), ctypes.byref(n)))
        ws = _device_bytes(n.value, probs.device)
        _check(L.tqc_topk_ws(*args, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
        ws.record_stream(_torch_stream(stream))
    return idx, val


def marginal(probs, num_qubits, keep, stream=None, workspace="torch"):
    """float64 marginal over the kept qubits (bit i of the result index =
    keep[i]); workspace as for topk."""
    if probs.numel() != (1 << int(num_qubits)):
        raise ValueError("probs must hold 2^num_qubits entries")
    out = torch.empty(1 << len(keep), dtype=torch.float64, device=probs.device)
    k = _i32arr(keep)
    L = lib()
    args = (ctypes.c_void_p(probs.data_ptr()), _dtype_code(probs), int(num_qubits), len(keep),
            ctypes.cast(k, _i32p), ctypes.c_void_p(out.data_ptr()))
    if workspace == "library":
        _check(L.tqc_marginal(*args, _stream_ptr(stream)))
    else:
        n = ctypes.c_uint64(0)
        _check(L.tqc_marginal_workspace_bytes(int(num_qubits), len(keep), ctypes.byref(n)))
        ws = _device_bytes(n.value, probs.device)
        _check(L.tqc_marginal_ws(*args, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
        ws.record_stream(_torch_stream(stream))
    return out


def _torch_stream(stream):
    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(stream))


class Batch:
    """Independent reconstructions run as one persistent, graph-captured launch."""

    def __init__(self, plans, outs=None, use_graph=True, grid=0, spin_limit=0, stream=None,
                 dependency_waits=False):
        L = lib()
        if outs is None:
            outs = [p.output_tensor() for p in plans]
        self.plans = list(plans)
        self.outs = list(outs)
        for p in self.plans:
            p._ready(stream)
        n = len(self.plans)
        ph = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        oh = (ctypes.c_void_p * n)(*[o.data_ptr() for o in self.outs])
        ob = (ctypes.c_uint64 * n)(*[o.numel() * o.element_size() for o in self.outs])
        opt = BatchOptions(int(bool(use_graph)), int(grid), int(bool(dependency_waits)),
                           int(spin_limit))
        h = ctypes.c_void_p()
        _check(L.tqc_batch_create(n, ph, oh, ob, ctypes.byref(opt), _stream_ptr(stream),
                                  ctypes.byref(h)))
        self.handle = h

    def execute(self, stream=None):
        _check(lib().tqc_batch_execute(self.handle, _stream_ptr(stream)))

    def execute_sequential(self, stream=None):
        n = len(self.plans)
        ms = (ctypes.c_double * (2 * n))()
        _check(lib().tqc_batch_execute_sequential(self.handle, _stream_ptr(stream),
                                                  ctypes.cast(ms, _dp)))
        return np.array(ms[:]).reshape(n, 2)

    def job_times(self):
        n = len(self.plans)
        a = (ctypes.c_double * n)()
        b = (ctypes.c_double * n)()
        err = ctypes.c_uint32()
        _check(lib().tqc_batch_job_times(self.handle, ctypes.cast(a, _dp), ctypes.cast(b, _dp),
                                         ctypes.byref(err)))
        return np.array(a[:]), np.array(b[:]), err.value

    def info(self):
        items = ctypes.c_uint64()
        units = ctypes.c_int32()
        grid = ctypes.c_int32()
        _check(lib().tqc_batch_info(self.handle, ctypes.byref(items), ctypes.byref(units),
                                    ctypes.byref(grid)))
        return {"items": items.value, "units": units.value, "grid": grid.value}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.tqc_batch_destroy(h)
            self.handle = None


class Multi:
    """Independent unsliced reconstructions replayed as one HIP graph
    (``use_graph``) or enqueued as plain launches, spread over ``streams``
    streams; ``streams=1, use_graph=False`` runs them one after another.
    ``grouped=True``: every kind of work of all jobs in shared launches, in
    ``waves`` waves; ``grouped="heads"``: only the launches before the
    pairwise steps shared (per wave), each job's pairwise steps and final
    step its own launches on ``streams`` worker streams.  Outputs equal each
    plan's own ``execute`` bit for bit."""

    def __init__(self, plans, outs=None, use_graph=True, streams=4, timed=False, stream=None,
                 grouped=False, waves=1):
        L = lib()
        if outs is None:
            outs = [p.output_tensor() for p in plans]
        self.plans = list(plans)
        self.outs = list(outs)
        self.timed = bool(timed)
        for p in self.plans:
            p._ready(stream)
        n = len(self.plans)
        ph = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        oh = (ctypes.c_void_p * n)(*[o.data_ptr() for o in self.outs])
        ob = (ctypes.c_uint64 * n)(*[o.numel() * o.element_size() for o in self.outs])
        h = ctypes.c_void_p()
        g = 2 if grouped == "heads" else int(bool(grouped))
        opt = MultiOptions(int(bool(use_graph)), int(streams), int(self.timed), g, int(waves))
        _check(L.tqc_multi_create_ex(n, ph, oh, ob, ctypes.byref(opt), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def execute(self, stream=None):
        _check(lib().tqc_multi_execute(self.handle, _stream_ptr(stream)))

    def info(self):
        """(launches per execute in grouped mode, else -1; final steps in
        shared persistent launches; those launches)."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().tqc_multi_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def job_times(self):
        """(start_ms, end_ms) per job, from the start of the last execute."""
        n = len(self.plans)
        a = (ctypes.c_double * n)()
        b = (ctypes.c_double * n)()
        _check(lib().tqc_multi_job_times(self.handle, ctypes.cast(a, _dp), ctypes.cast(b, _dp)))
        return np.array(a[:]), np.array(b[:])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.tqc_multi_destroy(h)
            self.handle = None


def find_cuts(num_qubits, gates, w_max, s_max, k_t=10, q_max=1e4):
    """Greedy graph growing cut search (Alg. 2-3): gates is a sequence of
    qubit tuples in circuit order; returns (labels, num_parts) with labels[g]
    the partition of two-qubit gate g and -1 for single-qubit gates."""
    flat = []
    for qs in gates:
        flat += [int(qs[0]), int(qs[1]) if len(qs) == 2 else -1]
    g = _i32arr(flat if flat else [0])
    n = len(gates)
    labels = (ctypes.c_int32 * max(1, n))()
    parts = ctypes.c_int32()
    _check(lib().tqc_find_cuts(int(num_qubits), n, ctypes.cast(g, _i32p), int(w_max), int(s_max), int(k_t),
                               float(q_max), ctypes.cast(labels, _i32p), ctypes.byref(parts)))
    return np.array(labels[:n], dtype=np.int32), parts.value


def batch_validate(plans, out_bytes=None):
    """Host emulation of the batch launch of these plans (tqc_batch_validate):
    '' when every access stays in bounds, else the first violation."""
    n = len(plans)
    ph = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    ob = (ctypes.c_uint64 * n)(*out_bytes) if out_bytes is not None else None
    rep = ctypes.create_string_buffer(1024)
    st = lib().tqc_batch_validate(n, ph, ob, rep, 1024)
    if st not in (0, 8):
        _check(st)
    return rep.value.decode()


def autotune(plan, out=None, reps=3, stream=None):
    """Measure every tile shape per step; keep the fastest (also in the process table)."""
    if out is None:
        out = plan.output_tensor()
    plan._ready(stream)
    _check(lib().tqc_plan_autotune(plan.handle, ctypes.c_void_p(out.data_ptr()),
                                   out.numel() * out.element_size(), int(reps), _stream_ptr(stream)))
    return [s["tile"] for s in plan.steps]


def autotune_save(path):
    _check(lib().tqc_autotune_save(os.fsencode(path)))


def autotune_load(path):
    _check(lib().tqc_autotune_load(os.fsencode(path)))


_fp = ctypes.POINTER(ctypes.c_float)


def _f32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, a.ctypes.data_as(_fp)


class CostModel:
    """MLP cost model (16 -> 64 -> 64 -> 1) trained and evaluated on the GPU."""

    def __init__(self, seed=1, _handle=None):
        L = lib()
        if _handle is None:
            h = ctypes.c_void_p()
            _check(L.tqc_costmodel_create(int(seed), ctypes.byref(h)))
            _handle = h
        self.handle = _handle
        self.num_params = L.tqc_costmodel_num_params()
        self.num_features = L.tqc_costmodel_num_features()

    @property
    def params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        _check(lib().tqc_costmodel_get_params(self.handle, out.ctypes.data_as(_fp), self.num_params))
        return out

    @params.setter
    def params(self, v):
        a, p = _f32(v)
        _check(lib().tqc_costmodel_set_params(self.handle, p, len(a)))

    def forward(self, X, stream=None):
        X, xp = _f32(X)
        y = np.empty(X.shape[0], dtype=np.float32)
        _check(lib().tqc_costmodel_forward(self.handle, xp, X.shape[0], y.ctypes.data_as(_fp),
                                           _stream_ptr(stream)))
        return y

    def gradients(self, X, t, stream=None):
        X, xp = _f32(X)
        t, tp = _f32(t)
        g = np.empty(self.num_params, dtype=np.float32)
        _check(lib().tqc_costmodel_gradients(self.handle, xp, tp, X.shape[0], g.ctypes.data_as(_fp),
                                             _stream_ptr(stream)))
        return g

    def train(self, feats, seconds, epochs=200, batch=256, lr=3e-3, seed=7, stream=None):
        F, fp = _f32(feats)
        T, tp = _f32(seconds)
        losses = np.empty(epochs, dtype=np.float32)
        o = TrainOptions(int(epochs), int(batch), float(lr), int(seed))
        _check(lib().tqc_costmodel_train(self.handle, fp, tp, F.shape[0], ctypes.byref(o),
                                         losses.ctypes.data_as(_fp), _stream_ptr(stream)))
        return losses

    def predict(self, feats, stream=None):
        F, fp = _f32(feats)
        out = np.empty(F.shape[0], dtype=np.float64)
        _check(lib().tqc_costmodel_predict(self.handle, fp, F.shape[0], out.ctypes.data_as(_dp),
                                           _stream_ptr(stream)))
        return out

    def save(self, path):
        _check(lib().tqc_costmodel_save(self.handle, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        _check(lib().tqc_costmodel_load(os.fsencode(path), ctypes.byref(h)))
        return cls(_handle=h)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            _LIB.tqc_costmodel_destroy(h)
            self.handle = None


def step_features(plan):
    """Raw feature rows (num_steps x 16) of a plan's contraction launches."""
    n = plan.stats["num_steps"]
    out = np.zeros((max(1, n), 16), dtype=np.float32)
    _check(lib().tqc_plan_step_features(plan.handle, out.ctypes.data_as(_fp), max(1, n)))
    return out[:n]
