// C-ABI of the tqc library: network validation, plan creation, execution
// and output forms.  Every entry point converts internal failures into a
// tqc_status and a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "device.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace tqc {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(tqc_status st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error{st, std::string(buf)};
}

#define HIP_OK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      tqc::fail(e_ == hipErrorOutOfMemory ? TQC_ERR_OUT_OF_MEMORY : TQC_ERR_DEVICE,       \
                "%s failed: %s", #expr, hipGetErrorString(e_));                           \
    }                                                                                     \
  } while (0)

template <typename F>
static tqc_status guarded(F &&f) {
  try {
    f();
    return TQC_OK;
  } catch (const Error &e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return TQC_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_last_error("internal error");
    return TQC_ERR_INTERNAL;
  }
}

Network::~Network() {
  for (auto &t : this->t) {
    if (t.dev_raw) (void)hipFree(t.dev_raw);
    t.dev_raw = nullptr;
  }
}

Plan::~Plan() {
  if (ws) (void)hipFree(ws);
  if (acc64) (void)hipFree(acc64);
}

// ------------------------------------------------------------ network
static Network *create_network(int32_t n, int32_t m, const tqc_tensor_desc *td, int32_t K,
                               const tqc_cut *cuts) {
  if (n < 0 || n > 4096) fail(TQC_ERR_INVALID_ARG, "num_qubits %d", n);
  if (m < 1 || !td) fail(TQC_ERR_INVALID_ARG, "need at least one tensor");
  if (K < 0 || (K > 0 && !cuts)) fail(TQC_ERR_INVALID_ARG, "cuts");
  std::unique_ptr<Network> net(new Network());
  net->n = n;
  net->m = m;
  net->K = K;
  net->cuts.assign(cuts, cuts + K);
  for (int c = 0; c < K; ++c) {
    const tqc_cut &e = net->cuts[c];
    if (e.upstream < 0 || e.upstream >= m || e.downstream < 0 || e.downstream >= m)
      fail(TQC_ERR_TOPOLOGY, "cut %d names tensor out of range", c);
    if (e.upstream == e.downstream)
      fail(TQC_ERR_TOPOLOGY, "cut %d joins tensor %d to itself", c, e.upstream);
  }
  std::vector<int> owner(n, -1);
  std::vector<std::vector<int>> cut_seen(K);
  net->t.resize(m);
  for (int j = 0; j < m; ++j) {
    const tqc_tensor_desc &d = td[j];
    TensorIn &t = net->t[j];
    if (d.num_cuts < 0 || d.num_outputs < 0 || (d.num_cuts && !d.cut_ids) ||
        (d.num_outputs && !d.output_qubits) || !d.data)
      fail(TQC_ERR_INVALID_ARG, "tensor %d descriptor", j);
    if (d.basis != TQC_BASIS_RAW && d.basis != TQC_BASIS_PAULI)
      fail(TQC_ERR_INVALID_ARG, "tensor %d basis", j);
    t.basis = d.basis;
    for (int i = 0; i < d.num_cuts; ++i) {
      int c = d.cut_ids[i];
      if (c < 0 || c >= K) fail(TQC_ERR_TOPOLOGY, "tensor %d lists cut %d out of range", j, c);
      if (std::find(t.cuts.begin(), t.cuts.end(), c) != t.cuts.end())
        fail(TQC_ERR_TOPOLOGY, "tensor %d lists cut %d twice", j, c);
      if (net->cuts[c].upstream != j && net->cuts[c].downstream != j)
        fail(TQC_ERR_TOPOLOGY, "tensor %d lists cut %d but is not one of its ends", j, c);
      t.cuts.push_back(c);
      t.up.push_back(net->cuts[c].upstream == j ? 1 : 0);
      cut_seen[c].push_back(j);
    }
    for (int i = 0; i < d.num_outputs; ++i) {
      int q = d.output_qubits[i];
      if (q < 0 || q >= n) fail(TQC_ERR_TOPOLOGY, "tensor %d output qubit %d out of range", j, q);
      if (owner[q] >= 0) fail(TQC_ERR_TOPOLOGY, "qubit %d is an output of tensors %d and %d", q, owner[q], j);
      owner[q] = j;
      t.outputs.push_back(q);
    }
    const int c = (int)t.cuts.size(), o = (int)t.outputs.size();
    if (2 * c + o > 44) fail(TQC_ERR_UNSUPPORTED, "tensor %d has 2^%d entries", j, 2 * c + o);
    t.u = 0;
    for (int x : t.up) t.u += x;
    t.d = c - t.u;
    if (t.basis == TQC_BASIS_PAULI) {
      t.rows = 1ull << (2 * c);
      t.cols = 1ull << o;
    } else {
      if (c > kMaxCutsT) fail(TQC_ERR_UNSUPPORTED, "raw tensor %d has more than %d cuts", j, kMaxCutsT);
      uint64_t r = 1;
      for (int x : t.up) r *= x ? 3 : 4;
      t.rows = r;
      t.cols = 1ull << (o + t.u);
    }
    const uint64_t cnt = t.rows * t.cols;
    t.host.assign(d.data, d.data + cnt);
    double mx = 0;
    for (double v : t.host) {
      if (!std::isfinite(v)) fail(TQC_ERR_INVALID_ARG, "tensor %d holds a non-finite value", j);
      mx = std::max(mx, std::fabs(v));
    }
    t.maxabs = mx;
  }
  for (int q = 0; q < n; ++q)
    if (owner[q] < 0) fail(TQC_ERR_TOPOLOGY, "qubit %d is not an output of any tensor", q);
  for (int c = 0; c < K; ++c)
    if (cut_seen[c].size() != 2)
      fail(TQC_ERR_TOPOLOGY, "cut %d appears in %zu tensor cut lists (needs its two ends)", c,
           cut_seen[c].size());
  return net.release();
}

static void upload(Network *net) {
  if (net->uploaded) return;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  for (auto &t : net->t) {
    const uint64_t bytes = t.rows * t.cols * 8;
    HIP_OK(hipMalloc((void **)&t.dev_raw, bytes ? bytes : 8));
    HIP_OK(hipMemcpy(t.dev_raw, t.host.data(), bytes, hipMemcpyHostToDevice));
  }
  net->device = dev;
  net->uploaded = true;
}

static void check_device(int want) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev != want) fail(TQC_ERR_INVALID_ARG, "current device %d, network lives on device %d", dev, want);
}

// --------------------------------------------------------------- execute
static void transform_tensor(const TensorIn &t, double *out, hipStream_t s) {
  TransformArgs a{};
  a.raw = t.dev_raw;
  a.out = out;
  a.c = (int)t.cuts.size();
  a.o = (int)t.outputs.size();
  a.u = t.u;
  uint64_t w = 1;
  for (int i = a.c - 1; i >= 0; --i) {
    a.up[i] = t.up[i];
    a.w[i] = w;
    w *= t.up[i] ? 3 : 4;
  }
  int bi = 0;
  for (int i = 0; i < a.c; ++i) a.bbit[i] = t.up[i] ? bi++ : -1;
  HIP_OK(launch_transform(a, s));
}

static void ensure_workspace(Plan *p, hipStream_t s) {
  Network *net = p->net;
  upload(net);
  check_device(net->device);
  if (!p->ws && p->ws_bytes) {
    HIP_OK(hipMalloc(&p->ws, p->ws_bytes));
    // operand padding beyond K is never written and must read as zero
    HIP_OK(hipMemsetAsync(p->ws, 0, p->ws_bytes, s));
  }
  // the Pauli tensors: raw ones are transformed into the workspace head
  uint64_t off = 0;
  for (auto &t : net->t) {
    if (t.basis == TQC_BASIS_RAW) {
      t.dev_pauli = (double *)((char *)p->ws + off);
      off = (off + t.pauli_entries() * 8 + 255) & ~uint64_t(255);
    } else {
      t.dev_pauli = t.dev_raw;
    }
  }
}

static int out_kind_for(Prec p) {
  switch (p) {
    case Prec::F64: return OUT_F64;
    case Prec::F32: return OUT_F32;
    case Prec::BF16X3: return OUT_SPLIT2;
    default: return OUT_SPLIT3;
  }
}

static void pack_leaf(Plan *p, int j, void *dst0, void *dst1, void *dst2, int prec_code,
                      uint64_t slice, hipStream_t s) {
  Network &net = *p->net;
  const TensorIn &t = net.t[j];
  const Node &nd = p->nodes[j];
  const int c = (int)t.cuts.size(), o = (int)t.outputs.size();
  PackArgs a{};
  a.src = t.dev_pauli;
  a.dst0 = dst0;
  a.dst1 = dst1;
  a.dst2 = dst2;
  a.prec = prec_code;
  a.scale = 1.0;
  a.nbits = (int)nd.labels.size();
  a.lk = nd.log2k;
  a.kpad = nd.kpad_log2;
  if (a.nbits > kMaxBits) fail(TQC_ERR_UNSUPPORTED, "operand with %d index bits", a.nbits);
  uint64_t base = 0;
  for (int i = 0; i < c; ++i) {
    const int cut = t.cuts[i];
    auto it = std::find(p->sliced.begin(), p->sliced.end(), cut);
    if (it != p->sliced.end()) {
      const int si = int(it - p->sliced.begin());
      const uint64_t digit = (slice >> (2 * si)) & 3;
      base |= digit << (o + 2 * (c - 1 - i));
    }
  }
  for (int i = 0; i < o; ++i) {
    auto it = std::find(p->fixed_q.begin(), p->fixed_q.end(), t.outputs[i]);
    if (it != p->fixed_q.end()) base |= (uint64_t)p->fixed_v[it - p->fixed_q.begin()] << i;
  }
  a.base = base;
  for (int i = 0; i < a.nbits; ++i) {
    const int l = nd.labels[i];
    if (l < 2 * net.K) {
      const int cut = l / 2, b = l % 2;
      const int li = int(std::find(t.cuts.begin(), t.cuts.end(), cut) - t.cuts.begin());
      a.inpos[i] = o + 2 * (c - 1 - li) + b;
    } else {
      const int q = l - 2 * net.K;
      a.inpos[i] = int(std::find(t.outputs.begin(), t.outputs.end(), q) - t.outputs.begin());
    }
  }
  HIP_OK(launch_pack(a, s));
}

static int pick_tile(const Plan *p, const Step &st) {
  (void)p;
  const int lmn = std::min(st.lm, st.ln);
  if (lmn >= 7) return 0;
  if (lmn >= 6) return 1;
  return 2;
}

// Per-phase timing with HIP events on the execution stream: phase 0 is the
// Pauli transform, 1 operand packing, 2 + i pairwise step i, then the final
// conversion.  Durations of a phase are summed over slices.
struct Timing {
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  hipStream_t s;
  int open_phase = -1;
  hipEvent_t open_ev = nullptr;
  void begin(int phase) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    HIP_OK(hipEventRecord(e, s));
    open_phase = phase;
    open_ev = e;
  }
  void end() {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    HIP_OK(hipEventRecord(e, s));
    ev.push_back({open_phase, {open_ev, e}});
    open_ev = nullptr;
  }
  void collect(double *ms, int nphases) {
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < nphases; ++i) ms[i] = 0.0;
    for (auto &x : ev) {
      float t = 0;
      HIP_OK(hipEventElapsedTime(&t, x.second.first, x.second.second));
      if (x.first < nphases) ms[x.first] += t;
    }
  }
  ~Timing() {
    for (auto &x : ev) {
      (void)hipEventDestroy(x.second.first);
      (void)hipEventDestroy(x.second.second);
    }
    if (open_ev) (void)hipEventDestroy(open_ev);
  }
};

// run slices [s0, s1); root output goes to `root_out` (dtype per kind)
static void run_slices(Plan *p, void *root_out, int root_kind, uint64_t s0, uint64_t s1,
                       bool accumulate_first, hipStream_t s, Timing *tm = nullptr) {
  Network &net = *p->net;
  const int m = net.m;
  const int pc = int(p->prec);
  const double scale = std::ldexp(1.0, -net.K);
  if (tm) tm->begin(0);
  for (auto &t : net.t)
    if (t.basis == TQC_BASIS_RAW) transform_tensor(t, t.dev_pauli, s);
  if (tm) tm->end();
  if (m == 1) {
    // a single tensor: its (fixed-qubit) slice is the output
    const int prec_code = root_kind == OUT_F64 || root_kind == OUT_F64_ACC ? 0 : 1;
    if (root_kind == OUT_F64_ACC) fail(TQC_ERR_UNSUPPORTED, "accumulating run of a single tensor");
    pack_leaf(p, 0, root_out, nullptr, nullptr, prec_code, 0, s);
    return;
  }
  bool first_done = false;
  for (uint64_t sl = s0; sl < s1; ++sl) {
    const bool first = (sl == s0);
    if (tm) tm->begin(1);
    for (int j = 0; j < m; ++j) {
      Node &nd = p->nodes[j];
      if (!first && !nd.slice_dep) continue;
      char *b = (char *)p->ws + nd.offset;
      pack_leaf(p, j, b, nd.planes > 1 ? b + nd.plane_bytes : nullptr,
                nd.planes > 2 ? b + 2 * nd.plane_bytes : nullptr, pc, sl, s);
    }
    if (tm) tm->end();
    for (size_t si = 0; si < p->steps.size(); ++si) {
      const Step &st = p->steps[si];
      Node &on = p->nodes[st.out];
      if (!first && !on.slice_dep) continue;
      const Node &na = p->nodes[st.a], &nb = p->nodes[st.b];
      GemmArgs g{};
      char *pa = (char *)p->ws + na.offset, *pb = (char *)p->ws + nb.offset;
      g.a0 = pa;
      g.a1 = na.planes > 1 ? pa + na.plane_bytes : nullptr;
      g.a2 = na.planes > 2 ? pa + 2 * na.plane_bytes : nullptr;
      g.b0 = pb;
      g.b1 = nb.planes > 1 ? pb + nb.plane_bytes : nullptr;
      g.b2 = nb.planes > 2 ? pb + 2 * nb.plane_bytes : nullptr;
      g.lm = st.lm;
      g.ln = st.ln;
      g.lk = st.lk;
      g.kpad = st.kpad_log2;
      if (st.lm > kMaxBits || st.ln > kMaxBits) fail(TQC_ERR_UNSUPPORTED, "step too large");
      for (int i = 0; i < st.lm; ++i) g.posM[i] = (uint8_t)st.posM[i];
      for (int i = 0; i < st.ln; ++i) g.posN[i] = (uint8_t)st.posN[i];
      if (st.root) {
        g.c0 = root_out;
        g.scale = scale;
        g.out_kind = root_kind;
        if (root_kind == OUT_F64_ACC && !accumulate_first && !first_done) g.out_kind = OUT_F64;
      } else {
        char *po = (char *)p->ws + on.offset;
        g.c0 = po;
        g.c1 = on.planes > 1 ? po + on.plane_bytes : nullptr;
        g.c2 = on.planes > 2 ? po + 2 * on.plane_bytes : nullptr;
        g.scale = 1.0;
        g.out_kind = out_kind_for(p->prec);
      }
      if (tm) tm->begin(2 + (int)si);
      HIP_OK(launch_gemm(pc, g, st.tile, s));
      if (tm) tm->end();
    }
    first_done = true;
  }
}

static void execute(Plan *p, void *out, uint64_t out_bytes, hipStream_t s, Timing *tm = nullptr) {
  const uint64_t entries = 1ull << p->out_bits;
  const uint64_t need = entries * (p->out_dtype == TQC_F64 ? 8 : 4);
  if (!out) fail(TQC_ERR_INVALID_ARG, "output pointer is null");
  if (out_bytes < need) fail(TQC_ERR_SHAPE, "output holds %llu bytes, needs %llu",
                             (unsigned long long)out_bytes, (unsigned long long)need);
  ensure_workspace(p, s);
  if (p->num_slices == 1) {
    run_slices(p, out, p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32, 0, 1, false, s, tm);
    return;
  }
  if (p->out_dtype == TQC_F64) {
    run_slices(p, out, OUT_F64_ACC, 0, p->num_slices, false, s, tm);
  } else {
    if (!p->acc64) HIP_OK(hipMalloc((void **)&p->acc64, entries * 8));
    run_slices(p, p->acc64, OUT_F64_ACC, 0, p->num_slices, false, s, tm);
    if (tm) tm->begin(2 + (int)p->steps.size());
    HIP_OK(launch_f64_to_f32(p->acc64, (float *)out, entries, s));
    if (tm) tm->end();
  }
}

// ----------------------------------------------------------- scratch
struct Scratch {
  std::mutex mu;
  void *ptr = nullptr;
  uint64_t bytes = 0;
  int device = -1;
};
static Scratch g_scratch;

static void *get_scratch(uint64_t bytes, hipStream_t s) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (g_scratch.ptr && (g_scratch.bytes < bytes || g_scratch.device != dev)) {
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipFree(g_scratch.ptr));
    g_scratch.ptr = nullptr;
  }
  if (!g_scratch.ptr) {
    HIP_OK(hipMalloc(&g_scratch.ptr, bytes));
    g_scratch.bytes = bytes;
    g_scratch.device = dev;
  }
  return g_scratch.ptr;
}

}  // namespace tqc

using namespace tqc;

struct tqc_network_s : Network {};
struct tqc_plan_s : Plan {};

extern "C" {

tqc_status tqc_network_create(int32_t num_qubits, int32_t num_tensors, const tqc_tensor_desc *tensors,
                              int32_t num_cuts, const tqc_cut *cuts, tqc_network_t *out) {
  return guarded([&] {
    if (!out) fail(TQC_ERR_INVALID_ARG, "out handle is null");
    *out = nullptr;
    Network *n = create_network(num_qubits, num_tensors, tensors, num_cuts, cuts);
    *out = reinterpret_cast<tqc_network_t>(n);
  });
}

tqc_status tqc_network_upload(tqc_network_t net) {
  return guarded([&] {
    if (!net) fail(TQC_ERR_INVALID_ARG, "null network");
    upload(reinterpret_cast<Network *>(net));
  });
}

void tqc_network_destroy(tqc_network_t net) { delete reinterpret_cast<Network *>(net); }

void tqc_plan_options_default(tqc_plan_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = TQC_FP32;
  o->out_dtype = TQC_F32;
  o->num_sliced = -1;
  o->cost_kind = TQC_COST_FLOPBYTE;
}

tqc_status tqc_plan_create(tqc_network_t net, const tqc_plan_options *opt, tqc_plan_t *out) {
  return guarded([&] {
    if (!net || !opt || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    Plan *p = build_plan(reinterpret_cast<Network *>(net), *opt);
    for (Step &st : p->steps) st.tile = pick_tile(p, st);
    *out = reinterpret_cast<tqc_plan_t>(p);
  });
}

void tqc_plan_destroy(tqc_plan_t plan) { delete reinterpret_cast<Plan *>(plan); }

tqc_status tqc_plan_get_stats(tqc_plan_t plan, tqc_plan_stats *st) {
  return guarded([&] {
    if (!plan || !st) fail(TQC_ERR_INVALID_ARG, "null argument");
    *st = reinterpret_cast<Plan *>(plan)->stats;
  });
}

tqc_status tqc_plan_get_step(tqc_plan_t plan, int32_t step, tqc_step_info *info) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !info) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (step < 0 || step >= (int)p->steps.size()) fail(TQC_ERR_INVALID_ARG, "step %d", step);
    const Step &s = p->steps[step];
    info->lhs = s.a;
    info->rhs = s.b;
    info->result = s.out;
    info->log2_m = s.lm;
    info->log2_n = s.ln;
    info->log2_k = s.lk;
    info->shared_cuts = s.lk / 2;
    info->open_cuts = 0;
    for (int l : s.m_labels) if (l < 2 * p->net->K) ++info->open_cuts;
    for (int l : s.n_labels) if (l < 2 * p->net->K) ++info->open_cuts;
    info->open_cuts /= 2;
    info->slice_dependent = p->nodes[s.out].slice_dep ? 1 : 0;
    info->tile = s.tile;
    info->flops = s.flops;
    info->bytes = s.bytes;
  });
}

tqc_status tqc_plan_get_sliced(tqc_plan_t plan, int32_t *cuts_out) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) fail(TQC_ERR_INVALID_ARG, "null plan");
    if (!p->sliced.empty() && !cuts_out) fail(TQC_ERR_INVALID_ARG, "null output");
    for (size_t i = 0; i < p->sliced.size(); ++i) cuts_out[i] = p->sliced[i];
  });
}

tqc_status tqc_execute(tqc_plan_t plan, void *out, uint64_t out_bytes, void *stream) {
  return guarded([&] {
    if (!plan) fail(TQC_ERR_INVALID_ARG, "null plan");
    execute(reinterpret_cast<Plan *>(plan), out, out_bytes, (hipStream_t)stream);
  });
}

tqc_status tqc_execute_profiled(tqc_plan_t plan, void *out, uint64_t out_bytes, void *stream,
                                double *phase_ms, int32_t num_phases) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !phase_ms) fail(TQC_ERR_INVALID_ARG, "null argument");
    const int need = 3 + (int)p->steps.size();
    if (num_phases < need) fail(TQC_ERR_SHAPE, "phase_ms needs %d entries", need);
    Timing tm;
    tm.s = (hipStream_t)stream;
    execute(p, out, out_bytes, (hipStream_t)stream, &tm);
    tm.collect(phase_ms, num_phases);
  });
}

tqc_status tqc_execute_slices(tqc_plan_t plan, double *out, uint64_t out_bytes, uint64_t slice_begin,
                              uint64_t slice_end, int32_t accumulate, void *stream) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    const uint64_t entries = 1ull << p->out_bits;
    if (out_bytes < entries * 8) fail(TQC_ERR_SHAPE, "output too small");
    if (slice_begin >= slice_end || slice_end > p->num_slices)
      fail(TQC_ERR_INVALID_ARG, "slice range [%llu, %llu) of %llu", (unsigned long long)slice_begin,
           (unsigned long long)slice_end, (unsigned long long)p->num_slices);
    if (p->net->m == 1) fail(TQC_ERR_UNSUPPORTED, "slice ranges need at least two tensors");
    ensure_workspace(p, (hipStream_t)stream);
    run_slices(p, out, OUT_F64_ACC, slice_begin, slice_end, accumulate != 0, (hipStream_t)stream);
  });
}

tqc_status tqc_network_pauli_tensor(tqc_network_t netp, int32_t j, double *out, uint64_t out_bytes,
                                    void *stream) {
  return guarded([&] {
    Network *net = reinterpret_cast<Network *>(netp);
    if (!net || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (j < 0 || j >= net->m) fail(TQC_ERR_INVALID_ARG, "tensor %d", j);
    upload(net);
    check_device(net->device);
    const TensorIn &t = net->t[j];
    const uint64_t bytes = t.pauli_entries() * 8;
    if (out_bytes < bytes) fail(TQC_ERR_SHAPE, "output too small");
    hipStream_t s = (hipStream_t)stream;
    if (t.basis == TQC_BASIS_PAULI)
      HIP_OK(hipMemcpyAsync(out, t.dev_raw, bytes, hipMemcpyDeviceToDevice, s));
    else
      transform_tensor(t, out, s);
  });
}

tqc_status tqc_topk(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k, uint64_t *idx_out,
                    double *val_out, void *stream) {
  return guarded([&] {
    if (!probs || !idx_out || !val_out) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (dtype != TQC_F32 && dtype != TQC_F64) fail(TQC_ERR_INVALID_ARG, "dtype");
    if (k < 1 || k > 4096 || (uint64_t)k > len) fail(TQC_ERR_INVALID_ARG, "k = %d for length %llu", k,
                                                     (unsigned long long)len);
    std::lock_guard<std::mutex> lk(g_scratch.mu);
    const uint64_t sb = topk_scratch_bytes(len, k);
    void *sp = get_scratch(sb, (hipStream_t)stream);
    HIP_OK(launch_topk(probs, dtype == TQC_F32 ? 1 : 0, len, k, idx_out, val_out, sp, sb,
                       (hipStream_t)stream));
  });
}

tqc_status tqc_marginal(const void *probs, tqc_dtype dtype, int32_t num_qubits, int32_t num_keep,
                        const int32_t *keep, double *out, void *stream) {
  return guarded([&] {
    if (!probs || !out || (num_keep > 0 && !keep)) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (dtype != TQC_F32 && dtype != TQC_F64) fail(TQC_ERR_INVALID_ARG, "dtype");
    if (num_qubits < 0 || num_qubits > 40) fail(TQC_ERR_INVALID_ARG, "num_qubits %d", num_qubits);
    if (num_keep < 0 || num_keep > 24 || num_keep > num_qubits)
      fail(TQC_ERR_INVALID_ARG, "num_keep %d", num_keep);
    for (int i = 0; i < num_keep; ++i) {
      if (keep[i] < 0 || keep[i] >= num_qubits) fail(TQC_ERR_INVALID_ARG, "keep qubit %d", keep[i]);
      for (int j = 0; j < i; ++j)
        if (keep[j] == keep[i]) fail(TQC_ERR_INVALID_ARG, "keep qubit %d twice", keep[i]);
    }
    std::lock_guard<std::mutex> lk(g_scratch.mu);
    const uint64_t sb = marginal_scratch_bytes(num_qubits, num_keep);
    void *sp = get_scratch(sb, (hipStream_t)stream);
    HIP_OK(launch_marginal(probs, dtype == TQC_F32 ? 1 : 0, num_qubits, num_keep, keep, out, sp, sb,
                           (hipStream_t)stream));
  });
}

const char *tqc_status_string(tqc_status s) {
  switch (s) {
    case TQC_OK: return "ok";
    case TQC_ERR_INVALID_ARG: return "invalid argument";
    case TQC_ERR_TOPOLOGY: return "invalid network topology";
    case TQC_ERR_SHAPE: return "shape or size mismatch";
    case TQC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case TQC_ERR_PLAN_INFEASIBLE: return "no plan fits the memory budget";
    case TQC_ERR_DEVICE: return "device error";
    case TQC_ERR_UNSUPPORTED: return "unsupported";
    case TQC_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char *tqc_last_error(void) { return g_last_error.c_str(); }

int32_t tqc_version(void) { return 100; }

}  // extern "C"
