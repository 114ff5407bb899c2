// C-ABI of the tqc library: network validation, plan creation, execution
// and output forms.  Every entry point converts internal failures into a
// tqc_status and a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <numeric>
#include <random>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "device.hpp"
#include "internal.hpp"
#include "transform_sched.hpp"
#include "batch.hpp"
#include "costmodel.hpp"
#include "dev_ops.hpp"
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
  if (ws_external) return;  // the caller's memory
  if (ws) (void)hipFree(ws);
  if (acc64) (void)hipFree(acc64);
  if (scale_buf) (void)hipFree(scale_buf);
  if (stats_buf) (void)hipFree(stats_buf);
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
static TransformArgs make_transform_args(const TensorIn &t, double *out);

// ------------------------------------------------- allocation-free top-k
// Scratch of tqc_topk_noalloc: a fixed device array, present on every GPU
// the library runs on for the life of the process.  Host code never uses
// the array's name as an address: the device address is looked up once per
// device with hipGetSymbolAddress and kept.
constexpr uint64_t kNoAllocScratchBytes = 8ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[64] = {};

static void *noalloc_scratch() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(TQC_ERR_UNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(TQC_ERR_DEVICE, "no device address for the top-k scratch on device %d", dev);
    g_noalloc_ptr[dev] = ptr;
  }
  return g_noalloc_ptr[dev];
}

// ---------------------------------------------------------- scratch
// Library-owned scratch of the calls that take no workspace argument
// (tqc_topk, tqc_marginal, tqc_network_pauli_tensor, heavy state selection,
// the standalone scans of a summary without a bound workspace): one buffer
// per (device, stream).  Work on one stream runs in order, so calls on that
// stream may reuse its buffer; calls on different streams never share one.
// The lease holds the buffer's lock while the call enqueues its kernels, so
// two host threads enqueuing on one stream do not interleave on it.  A
// buffer grows by synchronizing its stream and reallocating.
struct StreamScratch {
  std::mutex mu;
  void *ptr = nullptr;
  uint64_t bytes = 0;
};
struct ScratchLease {
  std::unique_lock<std::mutex> lock;
  void *ptr = nullptr;
};
static std::mutex g_scratch_map_mu;
static std::map<std::pair<int, hipStream_t>, std::unique_ptr<StreamScratch>> g_scratch_map;

static ScratchLease stream_scratch(uint64_t bytes, hipStream_t s) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  StreamScratch *e = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_map_mu);
    auto &slot = g_scratch_map[{dev, s}];
    if (!slot) slot.reset(new StreamScratch());
    e = slot.get();
  }
  ScratchLease l{std::unique_lock<std::mutex>(e->mu), nullptr};
  if (e->bytes < bytes) {
    if (e->ptr) {
      HIP_OK(hipStreamSynchronize(s));
      HIP_OK(hipFree(e->ptr));
      e->ptr = nullptr;
      e->bytes = 0;
    }
    HIP_OK(hipMalloc(&e->ptr, bytes ? bytes : 256));
    e->bytes = bytes;
  }
  l.ptr = e->ptr;
  return l;
}

// Separable transform of a raw tensor with at least kPassMinCuts cuts: each
// pass reads the previous layout and writes the next, alternating between
// two scratch buffers of `scr_bytes` each so that the last pass lands in dst.
// Appends pass i of the tensor to levels[i]; passes of one level (of
// different tensors) share a launch, and levels run in order.
// AbsMax (optional): the last pass also takes the abs-max of what it writes.
struct AbsMaxOut {
  unsigned long long *p = nullptr;
  uint64_t mask = 0, base = 0;
};

static void schedule_passes(const TensorIn &t, double *dst, double *s0, double *s1, uint64_t scr_bytes,
                            std::vector<std::vector<TransformPassArgs>> &levels, AbsMaxOut am = {}) {
  const TransformSchedule sc = transform_schedule(t);
  const int P = (int)sc.passes.size();
  if (P > 1 && sc.max_intermediate * 8 > scr_bytes) fail(TQC_ERR_INTERNAL, "transform scratch too small");
  if ((int)levels.size() < P) levels.resize(P);
  const double *in = t.dev_raw;
  for (int i = 0; i < P; ++i) {
    TransformPassArgs a = sc.passes[i];
    double *out = i == P - 1 ? dst : ((P - 2 - i) % 2 == 0 ? s0 : s1);
    a.in = in;
    a.out = out;
    if (i == P - 1) {
      a.amax = am.p;
      a.amask = am.mask;
      a.abase = am.base;
    }
    levels[i].push_back(a);
    in = out;
  }
}

// zero (optional): cleared by the first level's launch, which holds no
// tensor's last pass (every tensor on passes has at least two)
static void launch_levels(const std::vector<std::vector<TransformPassArgs>> &levels, hipStream_t s,
                          unsigned long long *zero = nullptr, int nzero = 0) {
  for (size_t L = 0; L < levels.size(); ++L) {
    if (L == 0 && zero)
      for (const auto &a : levels[0])
        if (a.amax) fail(TQC_ERR_INTERNAL, "a one-pass transform in the clearing launch");
    HIP_OK(launch_transform_passes(levels[L].data(), (int)levels[L].size(), s, L == 0 ? zero : nullptr,
                                   L == 0 ? nzero : 0));
  }
}

static void transform_tensor(const TensorIn &t, double *out, hipStream_t s) {
  if ((int)t.cuts.size() >= kPassMinCuts) {
    const uint64_t b = (transform_schedule(t).max_intermediate * 8 + 255) & ~uint64_t(255);
    ScratchLease lease = stream_scratch(2 * b, s);
    char *sp = (char *)lease.ptr;
    std::vector<std::vector<TransformPassArgs>> levels;
    schedule_passes(t, out, (double *)sp, (double *)(sp + b), b, levels);
    launch_levels(levels, s);
    return;
  }
  TransformArgs a = make_transform_args(t, out);
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
    case Prec::F16X3: return OUT_F32;  // pairwise steps in float32
    case Prec::BF16X3: return OUT_SPLIT2;
    default: return OUT_SPLIT3;
  }
}

// GEMM form of a step and pack form of the leaves: a float16-split plan runs
// its pairwise steps in float32 and only its final step on float16 planes
static int step_prec(const Plan *p, const Step &st) {
  if (p->prec != Prec::F16X3) return int(p->prec);
  return st.root ? 4 : 1;
}
static int pack_prec(const Plan *p) { return p->prec == Prec::F16X3 ? 1 : int(p->prec); }

// Tiling of a pack (PackArgs::tkb): the destination's lowest bits (k bits)
// and the source's lowest bits (output qubits) both in one LDS tile, when
// there are at least 2^2 and 2^3 of them: tkb = min(k bits, 5), tsb = the
// longest run of source positions 0, 1, ... gathered by destination bits
// above tkb, at most 10 - tkb.  Else tkb = 0 (one entry per thread).
static void set_pack_tiling(PackArgs &a) {
  a.tkb = a.tsb = 0;
  a.tmask = 0;
  const int kb = std::min(a.lk, 5);
  if (kb < 2) return;
  int sb = 0;
  int at[8];
  while (sb < 8 && kb + sb < 10) {
    int j = -1;
    for (int i = kb; i < a.nbits; ++i)
      if (a.inpos[i] == sb) j = i;
    if (j < 0) break;
    at[sb++] = j;
  }
  if (sb < 3) return;
  for (int i = 0; i < kb; ++i)
    if (a.inpos[i] < sb) return;  // a k bit among the source's lowest bits
  a.tkb = kb;
  a.tsb = sb;
  uint64_t in_tile = (1ull << kb) - 1;
  for (int q = 0; q < sb; ++q) {
    const int j = at[q];
    in_tile |= 1ull << j;
    a.dpos[q] = (int8_t)(j < a.lk ? j : j - a.lk + a.kpad);
  }
  a.tmask = ((a.nbits >= 64 ? ~0ull : (1ull << a.nbits) - 1)) & ~in_tile;
}

static PackArgs make_pack_args(Plan *p, int j, void *dst0, void *dst1, void *dst2, int prec_code,
                               uint64_t slice, const int *dexp = nullptr) {
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
  a.dexp = dexp;
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
  set_pack_tiling(a);
  return a;
}

static void pack_leaf(Plan *p, int j, void *dst0, void *dst1, void *dst2, int prec_code,
                      uint64_t slice, hipStream_t s, const int *dexp = nullptr) {
  PackArgs a = make_pack_args(p, j, dst0, dst1, dst2, prec_code, slice, dexp);
  HIP_OK(launch_pack(a, s));
}

// Exact power-of-two rescaling of the leaf operands: e_j makes the largest
// gathered |value| of leaf j (over all slices) lie in [1, 2); the final
// epilogue multiplies by 2^(-K - sum e_j) in float64.  Keeps float32 / bf16
// operands of many-factor networks away from underflow.
struct ScaleBuf {
  unsigned long long *maxbits;
  int *exps;
  double *root_scale;
  double *root_scale2;               // float16-split plans: root scale of the final step
  unsigned long long *maxbits16;     // ... and the abs-max of its two operands
};

static ScaleBuf scale_buffers(Plan *p) {
  const int m = p->net->m;
  if (!p->scale_buf) HIP_OK(hipMalloc(&p->scale_buf, 256 + (size_t)m * 16));
  char *b = (char *)p->scale_buf;
  return ScaleBuf{(unsigned long long *)(b + 256), (int *)(b + 256 + (size_t)m * 8), (double *)b, (double *)(b + 8),
                  (unsigned long long *)(b + 16)};
}

static AbsMaxArgs absmax_record(Plan *p, const ScaleBuf &sb, int j) {
  {
    const TensorIn &t = p->net->t[j];
    PackArgs pa = make_pack_args(p, j, nullptr, nullptr, nullptr, 0, 0);
    AbsMaxArgs a{};
    a.src = t.dev_pauli;
    a.base = 0;
    a.out = sb.maxbits + j;
    const int c = (int)t.cuts.size(), o = (int)t.outputs.size();
    for (int i = 0; i < o; ++i) {
      auto it = std::find(p->fixed_q.begin(), p->fixed_q.end(), t.outputs[i]);
      if (it != p->fixed_q.end()) a.base |= (uint64_t)p->fixed_v[it - p->fixed_q.begin()] << i;
    }
    a.nbits = pa.nbits;
    for (int i = 0; i < pa.nbits; ++i) a.inpos[i] = pa.inpos[i];
    for (int i = 0; i < c; ++i)
      if (std::find(p->sliced.begin(), p->sliced.end(), t.cuts[i]) != p->sliced.end()) {
        if (a.nbits + 2 > kMaxBits) fail(TQC_ERR_UNSUPPORTED, "operand with too many index bits");
        a.inpos[a.nbits++] = o + 2 * (c - 1 - i);
        a.inpos[a.nbits++] = o + 2 * (c - 1 - i) + 1;
      }
    // the maximum is the same in any visiting order: ascending source bit
    // positions make consecutive threads read consecutive addresses (the
    // packing order puts the cut digits, the slowest source bits, first)
    std::sort(a.inpos, a.inpos + a.nbits);
    return a;
  }
}

// The abs-max of leaf j as the transform that writes its Pauli tensor can
// take it: over the entries whose fixed output bits (the lowest bits of a
// Pauli index) hold their values.  Empty when leaf j's gathered entries are
// not exactly those, or it is not transformed.
static AbsMaxOut fused_absmax(Plan *p, const ScaleBuf &sb, int j) {
  const TensorIn &t = p->net->t[j];
  if (t.basis != TQC_BASIS_RAW) return {};
  const AbsMaxArgs a = absmax_record(p, sb, j);
  const int c = (int)t.cuts.size(), o = (int)t.outputs.size();
  AbsMaxOut am;
  int nfixed = 0;
  for (int i = 0; i < o; ++i)
    if (std::find(p->fixed_q.begin(), p->fixed_q.end(), t.outputs[i]) != p->fixed_q.end()) {
      am.mask |= 1ull << i;
      ++nfixed;
    }
  if (a.nbits != 2 * c + o - nfixed) return {};
  am.p = a.out;
  am.base = a.base;
  return am;
}

static TransformArgs make_transform_args(const TensorIn &t, double *out) {
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
  return a;
}

static int pick_tile(const Plan *p, const Step &st) {
  (void)p;
  const int lmn = std::min(st.lm, st.ln);
  if (lmn >= 7) return 0;
  if (lmn >= 6) return 1;
  return 2;
}

static GemmArgs make_gemm_args(Plan *p, const Step &st, void *root_out, int root_kind,
                               const double *dscale = nullptr) {
  const Node &na = p->nodes[st.a], &nb = p->nodes[st.b];
  const Node &on = p->nodes[st.out];
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
  if (p->splitk_bytes) {
    g.partial = (double *)((char *)p->ws + p->splitk_off);
    g.partial_bytes = p->splitk_bytes;
  }
  if (st.lm > kMaxBits || st.ln > kMaxBits) fail(TQC_ERR_UNSUPPORTED, "step too large");
  for (int i = 0; i < st.lm; ++i) g.posM[i] = (uint8_t)st.posM[i];
  for (int i = 0; i < st.ln; ++i) g.posN[i] = (uint8_t)st.posN[i];
  if (st.root && p->prec == Prec::F16X3) {
    char *ha = (char *)p->ws + p->h16_off[0], *hb = (char *)p->ws + p->h16_off[1];
    g.a0 = ha;
    g.a1 = ha + p->h16_plane[0];
    g.a2 = nullptr;
    g.b0 = hb;
    g.b1 = hb + p->h16_plane[1];
    g.b2 = nullptr;
    if (dscale) dscale = scale_buffers(p).root_scale2;
  }
  if (st.root) {
    g.c0 = root_out;
    g.scale = std::ldexp(1.0, -p->net->K);
    g.dscale = dscale;
    g.out_kind = root_kind;
  } else {
    char *po = (char *)p->ws + on.offset;
    g.c0 = po;
    g.c1 = on.planes > 1 ? po + on.plane_bytes : nullptr;
    g.c2 = on.planes > 2 ? po + 2 * on.plane_bytes : nullptr;
    g.scale = 1.0;
    g.out_kind = out_kind_for(p->prec);
  }
  return g;
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
// True when the plan's final step runs on the persistent final-step kernel
// (the same test run_slices applies before launching it).
static bool root_on_persistent(const Plan *p, const Step &st, const GemmArgs &g) {
  return st.root && st.tile == 0 && p->tile_policy != 2 && root_gemm_eligible(step_prec(p, st), g);
}

// The pairwise steps of one slice of a plan whose leaf operands are packed:
// every step for the first slice, only the slice-dependent ones after it.
// store_first: the final step stores where the run accumulates (its first
// slice of a float64 accumulation).
static void run_steps(Plan *p, void *root_out, int root_kind, const ScaleBuf &sb, bool first, bool store_first,
                      hipStream_t s, Timing *tm, unsigned long long *tkey, double *tsum, bool defer_root) {
  for (size_t si = 0; si < p->steps.size(); ++si) {
    const Step &st = p->steps[si];
    Node &on = p->nodes[st.out];
    if (!first && !on.slice_dep) continue;
    GemmArgs g = make_gemm_args(p, st, root_out, root_kind, sb.root_scale);
    if (st.root && store_first) g.out_kind = OUT_F64;
    if (st.root && tkey) {
      g.tkey = tkey;
      g.tsum = tsum;
    }
    if (tm) tm->begin(2 + (int)si);
    const int sp = step_prec(p, st);
    if (st.root && p->prec == Prec::F16X3) {
      // float32 operands of the final step -> two float16 planes each
      const Node &na = p->nodes[st.a], &nb = p->nodes[st.b];
      char *ha = (char *)p->ws + p->h16_off[0], *hb = (char *)p->ws + p->h16_off[1];
      HIP_OK(launch_f16_split((const float *)((char *)p->ws + na.offset), na.elems(), (uint16_t *)ha,
                              (uint16_t *)(ha + p->h16_plane[0]), (const float *)((char *)p->ws + nb.offset),
                              nb.elems(), (uint16_t *)hb, (uint16_t *)(hb + p->h16_plane[1]), sb.maxbits16,
                              sb.root_scale, sb.root_scale2, s));
    }
    if (root_on_persistent(p, st, g)) {
      // deferred: the caller runs it in a launch shared with other jobs
      if (!defer_root) HIP_OK(launch_root_gemm(sp, g, s));
    } else {
      HIP_OK(launch_gemm(sp, g, st.tile, s, p->tile_policy == 2));
    }
    if (tm) tm->end();
  }
}

static void run_slices(Plan *p, void *root_out, int root_kind, uint64_t s0, uint64_t s1,
                       bool accumulate_first, hipStream_t s, Timing *tm = nullptr,
                       unsigned long long *tkey = nullptr, double *tsum = nullptr, bool defer_root = false) {
  Network &net = *p->net;
  const int m = net.m;
  // operand scales (two or more tensors): the transform that writes a
  // leaf's Pauli tensor also takes its abs-max, and the first pack launch
  // turns the maxima into exponents and the output scale; a leaf given in
  // the Pauli basis gets an abs-max launch of its own
  const bool scaled = m >= 2;
  ScaleBuf sb{};
  if (scaled) sb = scale_buffers(p);
  std::vector<AbsMaxArgs> unfused;
  if (tm) tm->begin(0);
  {
    // tensors with several cuts: separable passes; the rest: the per-entry
    // kernel, up to four tensors per launch
    std::vector<TransformArgs> ta;
    std::vector<std::vector<TransformPassArgs>> levels;
    for (int j = 0; j < m; ++j) {
      TensorIn &t = net.t[j];
      const AbsMaxOut am = scaled ? fused_absmax(p, sb, j) : AbsMaxOut{};
      if (scaled && !am.p) unfused.push_back(absmax_record(p, sb, j));
      if (t.basis != TQC_BASIS_RAW) continue;
      if ((int)t.cuts.size() >= kPassMinCuts) {
        char *b = (char *)p->ws + p->tscr_off[j];
        schedule_passes(t, t.dev_pauli, (double *)b, (double *)(b + p->tscr_bytes[j]), p->tscr_bytes[j], levels,
                        am);
      } else {
        TransformArgs a = make_transform_args(t, t.dev_pauli);
        a.amax = am.p;
        a.amask = am.mask;
        a.abase = am.base;
        ta.push_back(a);
      }
    }
    // the maxima start from zero: cleared by the first pass level's launch,
    // else by a launch of their own, before any transform writes
    const bool fold = scaled && !levels.empty();
    if (scaled && !fold) HIP_OK(launch_zero_u64(sb.maxbits, (uint64_t)m, s));
    // the per-entry transforms join the last level's launch when it is not
    // the first (every tensor on passes has at least two) and both fit one
    const bool join = levels.size() >= 2 && !ta.empty() && ta.size() <= 4 &&
                      levels.back().size() <= (size_t)kPassBatch;
    if (join) {
      std::vector<TransformPassArgs> last = std::move(levels.back());
      levels.pop_back();
      launch_levels(levels, s, fold ? sb.maxbits : nullptr, fold ? m : 0);
      HIP_OK(launch_transform_level(last.data(), (int)last.size(), ta.data(), (int)ta.size(), s));
    } else {
      launch_levels(levels, s, fold ? sb.maxbits : nullptr, fold ? m : 0);
      if (!ta.empty()) HIP_OK(launch_transforms(ta.data(), (int)ta.size(), s));
    }
  }
  if (tm) tm->end();
  if (m == 1) {
    // a single tensor: its (fixed-qubit) slice is the output
    const int prec_code = root_kind == OUT_F64 || root_kind == OUT_F64_ACC ? 0 : 1;
    if (root_kind == OUT_F64_ACC) fail(TQC_ERR_UNSUPPORTED, "accumulating run of a single tensor");
    pack_leaf(p, 0, root_out, nullptr, nullptr, prec_code, 0, s);
    return;
  }
  bool first_done = false;
  if (!unfused.empty()) {
    if (tm) tm->begin(1);
    HIP_OK(launch_absmax(unfused.data(), (int)unfused.size(), s));
    if (tm) tm->end();
  }
  const ScaleRec sr{sb.maxbits, m, net.K, sb.exps, sb.root_scale};
  for (uint64_t sl = s0; sl < s1; ++sl) {
    const bool first = (sl == s0);
    if (tm) tm->begin(1);
    std::vector<PackArgs> packs;
    for (int j = 0; j < m; ++j) {
      Node &nd = p->nodes[j];
      if (!first && !nd.slice_dep) continue;
      char *b = (char *)p->ws + nd.offset;
      packs.push_back(make_pack_args(p, j, b, nd.planes > 1 ? b + nd.plane_bytes : nullptr,
                                     nd.planes > 2 ? b + 2 * nd.plane_bytes : nullptr, pack_prec(p), sl));
      packs.back().dmax = sb.maxbits + j;
    }
    if (!packs.empty()) HIP_OK(launch_packs(packs.data(), (int)packs.size(), s, first ? &sr : nullptr));
    if (tm) tm->end();
    const bool store_first = root_kind == OUT_F64_ACC && !accumulate_first && !first_done;
    run_steps(p, root_out, root_kind, sb, first, store_first, s, tm, tkey, tsum, defer_root);
    first_done = true;
  }
}

static void execute(Plan *p, void *out, uint64_t out_bytes, hipStream_t s, Timing *tm = nullptr,
                    bool defer_root = false) {
  const uint64_t entries = 1ull << p->out_bits;
  const uint64_t need = entries * (p->out_dtype == TQC_F64 ? 8 : 4);
  if (!out) fail(TQC_ERR_INVALID_ARG, "output pointer is null");
  if (out_bytes < need) fail(TQC_ERR_SHAPE, "output holds %llu bytes, needs %llu",
                             (unsigned long long)out_bytes, (unsigned long long)need);
  ensure_workspace(p, s);
  if (p->num_slices == 1) {
    run_slices(p, out, p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32, 0, 1, false, s, tm, nullptr, nullptr,
               defer_root);
    return;
  }
  if (p->out_dtype == TQC_F64) {
    run_slices(p, out, OUT_F64_ACC, 0, p->num_slices, false, s, tm);
  } else {
    if (!p->acc64) {
      if (p->ws_external) fail(TQC_ERR_SHAPE, "bound workspace has no float64 accumulator");
      HIP_OK(hipMalloc((void **)&p->acc64, entries * 8));
    }
    run_slices(p, p->acc64, OUT_F64_ACC, 0, p->num_slices, false, s, tm);
    if (tm) tm->begin(2 + (int)p->steps.size());
    HIP_OK(launch_f64_to_f32(p->acc64, (float *)out, entries, s));
    if (tm) tm->end();
  }
}

// The full vector plus its k largest entries and its float64 total.  A
// single-slice plan with at least two tensors gets them from per-tile
// statistics that the root contraction writes while storing its tiles (no
// extra pass over the 2^n output); otherwise the standalone scans run after
// the contraction.  Top-k results are identical either way; the totals differ
// only in float64 summation order.
// per-tile statistics of the root step (largest key and float64 sum, 16 B
// per tile) followed by the 256 float64 partial sums of their total
static uint64_t tile_stats_bytes(uint64_t ntiles) { return ((ntiles * 16 + 255) & ~uint64_t(255)) + 256 * 8; }

static const Step *root_step(const Plan *p) {
  for (const Step &st : p->steps)
    if (st.root) return &st;
  return nullptr;
}

static void execute_summary(Plan *p, void *out, uint64_t out_bytes, int k, uint64_t *idx_out,
                            double *val_out, double *total, hipStream_t s, Timing *tm) {
  const uint64_t entries = 1ull << p->out_bits;
  if (k < 0 || k > 4096 || (uint64_t)k > entries) fail(TQC_ERR_INVALID_ARG, "k = %d", k);
  if (!total || (k > 0 && (!idx_out || !val_out))) fail(TQC_ERR_INVALID_ARG, "null argument");
  const int dtype = p->out_dtype == TQC_F64 ? 0 : 1;
  const int fin_phase = 2 + (int)p->steps.size();
  const Step *root = nullptr;
  for (const Step &st : p->steps)
    if (st.root) root = &st;
  if (p->num_slices != 1 || p->net->m < 2 || !root) {
    execute(p, out, out_bytes, s, tm);
    const uint64_t sb = std::max(marginal_scratch_bytes(p->out_bits, 0),
                                 k > 0 ? topk_scratch_bytes(entries, k) : 0);
    ScratchLease lease;
    void *sp = p->scan_buf;
    if (!p->ws_external) {
      lease = stream_scratch(sb, s);
      sp = lease.ptr;
    } else if (p->scan_bytes < sb) {
      fail(TQC_ERR_SHAPE, "bound workspace has %llu scan bytes, needs %llu",
           (unsigned long long)p->scan_bytes, (unsigned long long)sb);
    }
    if (tm) tm->begin(fin_phase);
    HIP_OK(launch_marginal(out, dtype, p->out_bits, 0, nullptr, total, sp, sb, s));
    if (k > 0) HIP_OK(launch_topk(out, dtype, entries, k, idx_out, val_out, sp, sb, s));
    if (tm) tm->end();
    return;
  }
  const uint64_t need = entries * (p->out_dtype == TQC_F64 ? 8 : 4);
  if (!out) fail(TQC_ERR_INVALID_ARG, "output pointer is null");
  if (out_bytes < need) fail(TQC_ERR_SHAPE, "output holds %llu bytes, needs %llu",
                             (unsigned long long)out_bytes, (unsigned long long)need);
  ensure_workspace(p, s);
  const int bm = tile_bm(root->tile);
  const int lb = __builtin_ctz(bm);
  const uint64_t tilesM = ((1ull << root->lm) + bm - 1) / bm, tilesN = ((1ull << root->ln) + bm - 1) / bm;
  const uint64_t ntiles = tilesM * tilesN;
  const uint64_t tbytes = tile_stats_bytes(ntiles);
  const uint64_t sbytes = tbytes + topk_tiles_scratch_bytes(entries, ntiles, std::max(k, 1));
  if (p->stats_bytes < sbytes) {
    if (p->ws_external) fail(TQC_ERR_SHAPE, "bound workspace holds %llu statistics bytes, needs %llu",
                             (unsigned long long)p->stats_bytes, (unsigned long long)sbytes);
    if (p->stats_buf) {
      HIP_OK(hipStreamSynchronize(s));
      HIP_OK(hipFree(p->stats_buf));
      p->stats_buf = nullptr;
    }
    HIP_OK(hipMalloc(&p->stats_buf, sbytes));
    p->stats_bytes = sbytes;
  }
  unsigned long long *tkey = (unsigned long long *)p->stats_buf;
  double *tsum = (double *)(tkey + ntiles);
  char *tscratch = (char *)p->stats_buf + tbytes;
  run_slices(p, out, dtype == 0 ? OUT_F64 : OUT_F32, 0, 1, false, s, tm, tkey, tsum);
  GemmArgs g = make_gemm_args(p, *root, out, dtype == 0 ? OUT_F64 : OUT_F32);
  prepare_gemm_args(g, int(p->prec), bm, bm);  // compact tile order for the gather
  if (tm) tm->begin(fin_phase);
  HIP_OK(launch_sum_tiles(tsum, ntiles, (double *)(tscratch - 256 * 8), total, s));
  if (k > 0)
    HIP_OK(launch_topk_tiles(out, dtype, entries, g, lb, lb, tkey, ntiles, k, idx_out, val_out, tscratch,
                             sbytes - tbytes, s));
  if (tm) tm->end();
}

// ------------------------------------------------- caller-owned workspace
// One region holds every device buffer a plan uses, each 256-byte aligned:
//   [0, ws_bytes)  float64 Pauli tensors of raw inputs, transform ping-pong
//                  buffers, split-k partials, packed operands and
//                  intermediates, float16 planes (the planner's layout)
//   scale          per-leaf abs-max bits, exponents, output scales
//   acc            float64 accumulator of a sliced plan with float32 output
//   stats          single-slice plans of two or more tensors: the root's
//                  tile statistics plus the top-k gather scratch, sized for
//                  the smallest tile (32 x 32, so autotuning cannot outgrow
//                  it) and k = 4096
//   scan           other plans: the standalone top-k and total scans
struct PlanLayout {
  uint64_t scale_off = 0, acc_off = 0, acc_bytes = 0, stats_off = 0, stats_bytes = 0;
  uint64_t scan_off = 0, scan_bytes = 0, total = 0;
};

static PlanLayout plan_layout(const Plan *p) {
  auto al = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  const uint64_t entries = 1ull << p->out_bits;
  const int m = p->net->m;
  PlanLayout L;
  uint64_t off = al(p->ws_bytes);
  L.scale_off = off;
  off = al(off + 256 + (uint64_t)m * 16);
  if (p->num_slices > 1 && p->out_dtype == TQC_F32) {
    L.acc_off = off;
    L.acc_bytes = entries * 8;
    off = al(off + L.acc_bytes);
  }
  const Step *root = root_step(p);
  if (p->num_slices == 1 && m >= 2 && root) {
    const uint64_t ntiles = (((1ull << root->lm) + 31) / 32) * (((1ull << root->ln) + 31) / 32);
    L.stats_off = off;
    L.stats_bytes = al(tile_stats_bytes(ntiles) + topk_tiles_scratch_bytes(entries, ntiles, 4096));
    off += L.stats_bytes;
  } else {
    L.scan_off = off;
    L.scan_bytes = al(std::max(marginal_scratch_bytes(p->out_bits, 0), topk_scratch_bytes(entries, 4096)));
    off += L.scan_bytes;
  }
  L.total = off;
  return L;
}

// Point every device buffer of the plan into the caller's region (or, with
// ws = NULL, return to library-owned buffers allocated on first use).
// Library-owned buffers held so far are released first; hipFree waits for
// the device.  The region is cleared by a fill kernel on the stream: operand
// padding beyond K is never written and must read as zero.
static void bind_workspace(Plan *p, void *ws, uint64_t bytes, hipStream_t s) {
  if (!p->ws_external) {
    if (p->ws) HIP_OK(hipFree(p->ws));
    if (p->acc64) HIP_OK(hipFree(p->acc64));
    if (p->scale_buf) HIP_OK(hipFree(p->scale_buf));
    if (p->stats_buf) HIP_OK(hipFree(p->stats_buf));
  }
  p->ws = nullptr;
  p->acc64 = nullptr;
  p->scale_buf = nullptr;
  p->stats_buf = nullptr;
  p->stats_bytes = 0;
  p->scan_buf = nullptr;
  p->scan_bytes = 0;
  p->ws_external = false;
  if (!ws) return;
  const PlanLayout L = plan_layout(p);
  if ((uintptr_t)ws & 255) fail(TQC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    fail(TQC_ERR_SHAPE, "workspace holds %llu bytes, the plan needs %llu", (unsigned long long)bytes,
         (unsigned long long)L.total);
  upload(p->net);
  check_device(p->net->device);
  char *b = (char *)ws;
  p->ws = b;
  p->scale_buf = b + L.scale_off;
  p->acc64 = L.acc_bytes ? (double *)(b + L.acc_off) : nullptr;
  p->stats_buf = L.stats_bytes ? b + L.stats_off : nullptr;
  p->stats_bytes = L.stats_bytes;
  p->scan_buf = L.scan_bytes ? b + L.scan_off : nullptr;
  p->scan_bytes = L.scan_bytes;
  p->ws_external = true;
  HIP_OK(launch_zero_u64((unsigned long long *)b, L.total / 8, s));
}

// ------------------------------------------------------------------ batch
struct Batch {
  std::vector<Plan *> plans;
  std::vector<void *> outs;
  int prec = 1;
  int njobs = 0;
  int nunits = 0;
  int grid = 0;
  uint64_t total = 0;
  void *dmem = nullptr;  // one allocation for all tables and counters
  BatchDesc desc{};
  bool use_graph = true;
  int by_level = 1;
  std::vector<unsigned long long> level_first;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  double tick_khz = 100000.0;
  int device = -1;
  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (dmem) (void)hipFree(dmem);
  }
};

constexpr bool kBatchLaunchEnabled = false;

// Work tables of a batch: per-job pre-pass records (Pauli transform of raw
// tensors, leaf abs-max), pack and GEMM argument records, and the work units
// in level order with their item ranges.  Built from the plans' device
// pointers (workspaces, Pauli tensors, outputs); the device addresses of
// the batch's own buffers (leaf exponents, job scales, abs-max bits) are
// filled in later through `fixes`.
struct BatchTables {
  struct Fix { int kind; size_t idx; int leaf; int job; };
  std::vector<BatchUnit> fin;
  std::vector<TransformArgs> targs;
  std::vector<AbsMaxArgs> aargs;
  std::vector<PackArgs> pargs;
  std::vector<GemmArgs> gargs;
  std::vector<Fix> fixes;
  std::vector<int> job_leaf0{0}, job_cuts;
  std::vector<unsigned long long> level_first;
  uint64_t max_t = 0, max_l = 0, total = 0;
  int nleaves = 0;
};

static BatchTables build_batch_tables(int njobs, Plan *const *plans, void *const *outs, int prec) {
  BatchTables T;
  struct TmpUnit {
    BatchUnit u;
    int level;
    double cost;
  };
  std::vector<TmpUnit> units;
  for (int j = 0; j < njobs; ++j) {
    Plan *p = plans[j];
    Network &net = *p->net;
    const int m = net.m;
    const int root_kind = p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32;
    const double job_cost = p->stats.predicted_seconds;
    std::vector<int> node_unit(p->nodes.size(), -1), depth(p->nodes.size(), 0);
    for (int t = 0; t < m; ++t) {
      const TensorIn &ti = net.t[t];
      if (ti.basis != TQC_BASIS_RAW) continue;
      const TransformArgs ta = make_transform_args(ti, ti.dev_pauli);
      // the transform kernel's loop bounds: 4^c x 2^o entries, 2 bits of
      // option state per cut in 32 bits, raw rows x 2^(o+u) columns
      if (ta.c > kMaxCutsT || ta.o + ta.u > 62 || 2 * ta.c + ta.o > 62 || !ta.raw || !ta.out)
        fail(TQC_ERR_UNSUPPORTED, "job %d tensor %d: transform of %d cuts, %d outputs", j, t, ta.c, ta.o);
      uint64_t rows = 1;
      for (int i = 0; i < ta.c; ++i) rows *= ta.up[i] ? 3 : 4;
      if (rows != ti.rows || (1ull << (ta.o + ta.u)) != ti.cols)
        fail(TQC_ERR_INTERNAL, "job %d tensor %d: transform record does not match its raw layout", j, t);
      T.targs.push_back(ta);
      T.max_t = std::max<uint64_t>(T.max_t, ti.pauli_entries());
    }
    const int leaf0 = T.job_leaf0.back();
    if (m >= 2) {
      // abs-max of every leaf (its gathered entries, all slices)
      for (int t = 0; t < m; ++t) {
        const TensorIn &ti = net.t[t];
        PackArgs pa = make_pack_args(p, t, nullptr, nullptr, nullptr, 0, 0);
        AbsMaxArgs a{};
        a.src = ti.dev_pauli;
        const int o = (int)ti.outputs.size();
        for (int i = 0; i < o; ++i) {
          auto it = std::find(p->fixed_q.begin(), p->fixed_q.end(), ti.outputs[i]);
          if (it != p->fixed_q.end()) a.base |= (uint64_t)p->fixed_v[it - p->fixed_q.begin()] << i;
        }
        a.nbits = pa.nbits;
        for (int i = 0; i < pa.nbits; ++i) a.inpos[i] = pa.inpos[i];
        // largest source index the abs-max kernel forms: every gathered bit set
        uint64_t hi = a.base;
        for (int i = 0; i < a.nbits; ++i) hi += 1ull << a.inpos[i];
        if (a.nbits > kMaxBits || !a.src || hi >= ti.pauli_entries())
          fail(TQC_ERR_INTERNAL, "job %d leaf %d: abs-max reads index %llu of %llu", j, t, (unsigned long long)hi,
               (unsigned long long)ti.pauli_entries());
        T.fixes.push_back({0, T.aargs.size(), leaf0 + t, j});
        T.aargs.push_back(a);
        T.max_l = std::max<uint64_t>(T.max_l, 1ull << a.nbits);
      }
      T.job_leaf0.push_back(leaf0 + m);
    } else {
      T.job_leaf0.push_back(leaf0);
    }
    T.job_cuts.push_back(net.K);
    for (int t = 0; t < m; ++t) {
      const Node &nd = p->nodes[t];
      TmpUnit u{};
      u.u.kind = UNIT_PACK;
      u.u.job = j;
      u.u.dep0 = -1;
      u.u.dep1 = -1;
      u.u.arg = (int)T.pargs.size();
      if (m == 1) {
        T.pargs.push_back(make_pack_args(p, t, outs[j], nullptr, nullptr, p->out_dtype == TQC_F64 ? 0 : 1, 0));
        u.u.is_root = 1;
      } else {
        char *bp = (char *)p->ws + nd.offset;
        T.pargs.push_back(make_pack_args(p, t, bp, nd.planes > 1 ? bp + nd.plane_bytes : nullptr,
                                         nd.planes > 2 ? bp + 2 * nd.plane_bytes : nullptr, int(p->prec), 0));
        T.fixes.push_back({1, T.pargs.size() - 1, leaf0 + t, j});
      }
      u.u.ntiles = ((1ull << nd.labels.size()) + 4095) / 4096;
      u.level = 1;
      u.cost = job_cost;
      node_unit[t] = (int)units.size();
      units.push_back(u);
    }
    for (const Step &st : p->steps) {
      TmpUnit u{};
      u.u.kind = UNIT_GEMM;
      u.u.job = j;
      u.u.dep0 = node_unit[st.a];
      u.u.dep1 = node_unit[st.b];
      u.u.arg = (int)T.gargs.size();
      u.u.tile = st.tile;
      u.u.is_root = st.root ? 1 : 0;
      GemmArgs g = make_gemm_args(p, st, outs[j], root_kind);
      const int bm = tile_bm(st.tile);
      prepare_gemm_args(g, prec, bm, bm);
      g.swz = 0;  // the work queue decides placement
      if (st.root) T.fixes.push_back({2, T.gargs.size(), -1, j});
      T.gargs.push_back(g);
      const uint64_t tm = ((1ull << st.lm) + bm - 1) / bm, tn = ((1ull << st.ln) + bm - 1) / bm;
      u.u.ntiles = tm * tn;
      depth[st.out] = 1 + std::max(depth[st.a], depth[st.b]);
      u.level = 1 + depth[st.out];
      u.cost = job_cost;
      node_unit[st.out] = (int)units.size();
      units.push_back(u);
    }
  }
  T.nleaves = T.job_leaf0.back();
  // the pre-pass grids index records by blockIdx.y
  if (T.targs.size() > 65535 || T.nleaves > 65535) fail(TQC_ERR_UNSUPPORTED, "too many tensors in one batch");
  // level order; inside a level, the most expensive jobs first
  std::vector<int> order(units.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (units[x].level != units[y].level) return units[x].level < units[y].level;
    return units[x].cost > units[y].cost;
  });
  std::vector<int> newid(units.size());
  for (size_t i = 0; i < order.size(); ++i) newid[order[i]] = (int)i;
  T.fin.resize(units.size());
  uint64_t first = 0;
  for (size_t i = 0; i < order.size(); ++i) {
    BatchUnit u = units[order[i]].u;
    if (u.dep0 >= 0) u.dep0 = newid[u.dep0];
    if (u.dep1 >= 0) u.dep1 = newid[u.dep1];
    u.first = first;
    first += u.ntiles;
    T.fin[i] = u;
  }
  T.total = first;
  // item ranges of the levels (units are sorted by level)
  std::vector<int> lev(order.size());
  for (size_t i = 0; i < order.size(); ++i) lev[i] = units[order[i]].level;
  for (size_t i = 0; i < T.fin.size(); ++i)
    if (i == 0 || lev[i] != lev[i - 1]) T.level_first.push_back(T.fin[i].first);
  T.level_first.push_back(first);
  return T;
}

static Batch *create_batch(int njobs, Plan *const *plans, void *const *outs, const uint64_t *out_bytes,
                           const tqc_batch_options &opt, hipStream_t s) {
  if (njobs < 1) fail(TQC_ERR_INVALID_ARG, "no jobs");
  std::unique_ptr<Batch> b(new Batch());
  b->njobs = njobs;
  b->use_graph = opt.use_graph != 0;
  b->by_level = opt.dependency_waits ? 0 : 1;
  b->prec = int(plans[0]->prec);
  for (int j = 0; j < njobs; ++j) {
    Plan *p = plans[j];
    if (!p || !outs || !outs[j]) fail(TQC_ERR_INVALID_ARG, "job %d: null plan or output", j);
    if (int(p->prec) != b->prec) fail(TQC_ERR_INVALID_ARG, "job %d: all jobs need one precision", j);
    if (p->prec == Prec::F16X3) fail(TQC_ERR_UNSUPPORTED, "job %d: float16-split plans are not batched", j);
    if (p->num_slices != 1) fail(TQC_ERR_UNSUPPORTED, "job %d: sliced plans are not batched", j);
    const uint64_t need = (1ull << p->out_bits) * (p->out_dtype == TQC_F64 ? 8 : 4);
    if (out_bytes && out_bytes[j] < need) fail(TQC_ERR_SHAPE, "job %d: output too small", j);
    for (int i = 0; i < j; ++i)
      if (plans[i] == p || plans[i]->net == p->net)
        fail(TQC_ERR_INVALID_ARG, "jobs %d and %d share a plan or network", i, j);
    ensure_workspace(p, s);
    b->plans.push_back(p);
    b->outs.push_back(outs[j]);
  }
  BatchTables T = build_batch_tables(njobs, plans, outs, b->prec);
  std::vector<BatchUnit> &fin = T.fin;
  std::vector<TransformArgs> &targs = T.targs;
  std::vector<AbsMaxArgs> &aargs = T.aargs;
  std::vector<PackArgs> &pargs = T.pargs;
  std::vector<GemmArgs> &gargs = T.gargs;
  std::vector<int> &job_leaf0 = T.job_leaf0, &job_cuts = T.job_cuts;
  const int nleaves = T.nleaves;
  const uint64_t max_t = T.max_t, max_l = T.max_l;
  b->nunits = (int)fin.size();
  b->total = T.total;
  b->level_first = T.level_first;
  // host-side checks before anything runs: dependencies point backwards,
  // and every argument record is within the ranges the kernels assume
  for (size_t i = 0; i < fin.size(); ++i) {
    const BatchUnit &u = fin[i];
    if (u.dep0 >= (int)i || u.dep1 >= (int)i) fail(TQC_ERR_INTERNAL, "batch unit %zu depends forward", i);
    if (u.ntiles == 0) fail(TQC_ERR_INTERNAL, "batch unit %zu has no items", i);
    if (u.kind == UNIT_PACK) {
      const PackArgs &a = pargs[u.arg];
      if (a.nbits > kMaxBits || a.lk > a.kpad || a.kpad > 40 || !a.src || !a.dst0 ||
          u.ntiles != ((1ull << a.nbits) + 4095) / 4096)
        fail(TQC_ERR_INTERNAL, "batch pack unit %zu has bad arguments", i);
    } else {
      const GemmArgs &g = gargs[u.arg];
      const int bm = tile_bm(u.tile);
      const uint64_t tiles = (((1ull << g.lm) + bm - 1) / bm) * (((1ull << g.ln) + bm - 1) / bm);
      if (g.lm > kMaxBits || g.ln > kMaxBits || g.lk > g.kpad || g.kpad > 40 || g.kpad < 4 ||
          !g.a0 || !g.b0 || !g.c0 || u.ntiles != tiles || g.swz != 0)
        fail(TQC_ERR_INTERNAL, "batch gemm unit %zu has bad arguments", i);
    }
  }
  // one device allocation: units, args, counters, job clocks, flags
  auto al = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  uint64_t off = 0;
  const uint64_t o_units = off; off = al(off + fin.size() * sizeof(BatchUnit));
  const uint64_t o_t = off; off = al(off + std::max<size_t>(1, targs.size()) * sizeof(TransformArgs));
  const uint64_t o_p = off; off = al(off + pargs.size() * sizeof(PackArgs));
  const uint64_t o_g = off; off = al(off + std::max<size_t>(1, gargs.size()) * sizeof(GemmArgs));
  const uint64_t o_c = off; off = al(off + fin.size() * 4);
  const uint64_t o_n = off; off = al(off + 8 * (b->level_first.size() + 1));
  const uint64_t o_s = off; off = al(off + njobs * 8);
  const uint64_t o_e = off; off = al(off + njobs * 8);
  const uint64_t o_err = off; off = al(off + 4);
  const uint64_t o_a = off; off = al(off + std::max<size_t>(1, aargs.size()) * sizeof(AbsMaxArgs));
  const uint64_t o_mx = off; off = al(off + std::max(1, nleaves) * 8);
  const uint64_t o_ex = off; off = al(off + std::max(1, nleaves) * 4);
  const uint64_t o_rs = off; off = al(off + njobs * 8);
  const uint64_t o_l0 = off; off = al(off + (njobs + 1) * 4);
  const uint64_t o_k = off; off = al(off + njobs * 4);
  HIP_OK(hipMalloc(&b->dmem, off));
  char *dm = (char *)b->dmem;
  unsigned long long *d_max = (unsigned long long *)(dm + o_mx);
  int *d_exp = (int *)(dm + o_ex);
  double *d_rs = (double *)(dm + o_rs);
  for (const BatchTables::Fix &f : T.fixes) {
    if (f.kind == 0) aargs[f.idx].out = d_max + f.leaf;
    else if (f.kind == 1) pargs[f.idx].dexp = d_exp + f.leaf;
    else gargs[f.idx].dscale = d_rs + f.job;
  }
  if (!aargs.empty())
    HIP_OK(hipMemcpy(dm + o_a, aargs.data(), aargs.size() * sizeof(AbsMaxArgs), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dm + o_l0, job_leaf0.data(), (njobs + 1) * 4, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dm + o_k, job_cuts.data(), njobs * 4, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dm + o_units, fin.data(), fin.size() * sizeof(BatchUnit), hipMemcpyHostToDevice));
  if (!targs.empty())
    HIP_OK(hipMemcpy(dm + o_t, targs.data(), targs.size() * sizeof(TransformArgs), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dm + o_p, pargs.data(), pargs.size() * sizeof(PackArgs), hipMemcpyHostToDevice));
  if (!gargs.empty())
    HIP_OK(hipMemcpy(dm + o_g, gargs.data(), gargs.size() * sizeof(GemmArgs), hipMemcpyHostToDevice));
  BatchDesc &d = b->desc;
  d.units = (const BatchUnit *)(dm + o_units);
  d.nunits = b->nunits;
  d.targs = (const TransformArgs *)(dm + o_t);
  d.pargs = (const PackArgs *)(dm + o_p);
  d.gargs = (const GemmArgs *)(dm + o_g);
  d.counters = (unsigned int *)(dm + o_c);
  d.next = (unsigned long long *)(dm + o_n);
  d.total = b->total;
  d.job_start = (unsigned long long *)(dm + o_s);
  d.job_end = (unsigned long long *)(dm + o_e);
  d.error = (unsigned int *)(dm + o_err);
  d.spin_limit = opt.spin_limit ? opt.spin_limit : (1ull << 30);
  d.ntransforms = (int)targs.size();
  d.max_transform_elems = max_t;
  d.aargs = (const AbsMaxArgs *)(dm + o_a);
  d.nleaves = nleaves;
  d.max_leaf_elems = max_l;
  d.maxbits = d_max;
  d.exps = d_exp;
  d.root_scale = d_rs;
  d.job_leaf0 = (const int *)(dm + o_l0);
  d.job_cuts = (const int *)(dm + o_k);
  d.nlevels = (int)b->level_first.size() - 1;
  d.level_first = b->level_first.data();
  d.nowait = b->by_level;
  d.first_item = 0;
  int dev = 0, cus = 0, khz = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  b->device = dev;
  b->tick_khz = khz > 0 ? double(khz) : 100000.0;
  const int per_cu = batch_blocks_per_cu(b->prec);
  b->grid = opt.grid > 0 ? opt.grid : per_cu * cus;
  return b.release();
}

static void batch_execute(Batch *b, hipStream_t s) {
  // Switched off: runs of the persistent batch launch did not finish on
  // MI355X, and the cause has not been shown yet.
  if (!kBatchLaunchEnabled)
    fail(TQC_ERR_UNSUPPORTED, "persistent batch execution is switched off (a run did not finish and "
                              "its cause is not identified); use tqc_batch_execute_sequential");
  check_device(b->device);
  b->last_stream = s;
  if (!b->use_graph) {
    HIP_OK(launch_batch(b->prec, b->desc, b->njobs, b->grid, b->by_level, s));
    return;
  }
  if (!b->exec) {
    // capture reset + persistent launch once on a private stream
    HIP_OK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_batch(b->prec, b->desc, b->njobs, b->grid, b->by_level, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(b->cap_stream, &g);
    HIP_OK(le);
    HIP_OK(ce);
    b->graph = g;
    HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  HIP_OK(hipGraphLaunch(b->exec, s));
}

static void batch_sequential(Batch *b, hipStream_t s, double *job_ms) {
  check_device(b->device);
  std::vector<hipEvent_t> ev(2 * b->njobs);
  for (auto &e : ev) HIP_OK(hipEventCreate(&e));
  for (int j = 0; j < b->njobs; ++j) {
    Plan *p = b->plans[j];
    HIP_OK(hipEventRecord(ev[2 * j], s));
    execute(p, b->outs[j], ~0ull, s);
    HIP_OK(hipEventRecord(ev[2 * j + 1], s));
  }
  HIP_OK(hipStreamSynchronize(s));
  for (int j = 0; j < b->njobs; ++j) {
    float t0 = 0, t1 = 0;
    HIP_OK(hipEventElapsedTime(&t0, ev[0], ev[2 * j]));
    HIP_OK(hipEventElapsedTime(&t1, ev[0], ev[2 * j + 1]));
    if (job_ms) {
      job_ms[2 * j] = t0;
      job_ms[2 * j + 1] = t1;
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
}

static void batch_times(Batch *b, double *start_ms, double *end_ms, uint32_t *error) {
  HIP_OK(hipStreamSynchronize(b->last_stream));
  std::vector<unsigned long long> st(b->njobs), en(b->njobs);
  unsigned int err = 0;
  HIP_OK(hipMemcpy(st.data(), b->desc.job_start, b->njobs * 8, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(en.data(), b->desc.job_end, b->njobs * 8, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&err, b->desc.error, 4, hipMemcpyDeviceToHost));
  (void)0;
  unsigned long long t0 = ~0ull;
  for (auto x : st) t0 = std::min(t0, x);
  for (int j = 0; j < b->njobs; ++j) {
    if (start_ms) start_ms[j] = double(st[j] - t0) / b->tick_khz;
    if (end_ms) end_ms[j] = en[j] >= t0 ? double(en[j] - t0) / b->tick_khz : -1.0;
  }
  if (error) *error = err;
}

// ----------------------------------------------- host emulation of a batch
// Replays on the host what the batch launch would do for these plans, with
// no device work: the plans' and networks' device pointers are replaced by
// distinct synthetic addresses (each buffer its own region, far apart), the
// work tables are built exactly as for the launch, and then every kernel's
// loop bounds and every address it would read or write are walked:
//   pre-pass: the Pauli transform's option odometer per entry (iteration
//     count, raw reads, Pauli writes), every abs-max read, the exponent and
//     scale writes;
//   persistent part: every item's unit lookup (the kernel's binary search),
//     each pack chunk's reads and writes, each GEMM tile's operand rows and
//     k range against the tile's k step, its output addresses (direct, or
//     through the staged compact index, which must equal the direct ones),
//     and the level / dependency order of units.
// An access must stay inside the region of the pointer it is made through.
// Returns an empty string, or a description of the first violation.
namespace {
struct EmuRegions {
  struct R { uint64_t lo, hi; std::string what; };
  std::vector<R> r;
  uint64_t next = 1ull << 44;
  void *fresh(uint64_t bytes, const std::string &what) {
    const uint64_t lo = next;
    next += (((bytes + 4095) >> 12) << 12) + (1ull << 36);
    r.push_back({lo, lo + bytes, what});
    return (void *)lo;
  }
  void add(const void *p, uint64_t bytes, const std::string &what) {
    r.push_back({(uint64_t)p, (uint64_t)p + bytes, what});
  }
  const R *find(const void *p) const {
    const uint64_t a = (uint64_t)p;
    const R *best = nullptr;
    for (const R &x : r)
      if (a >= x.lo && a < x.hi + (x.hi == x.lo ? 1 : 0) && (!best || x.hi - x.lo < best->hi - best->lo)) best = &x;
    return best;
  }
};

struct EmuFail {
  std::string msg;
};

[[noreturn]] void emu_fail(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw EmuFail{buf};
}

void emu_access(const EmuRegions &R, const void *base, uint64_t elem, uint64_t esz, const char *what) {
  const EmuRegions::R *reg = R.find(base);
  if (!reg) emu_fail("%s: pointer %p lies in no buffer", what, base);
  const uint64_t a = (uint64_t)base + elem * esz;
  if (a < reg->lo || a + esz > reg->hi)
    emu_fail("%s: element %llu (%llu bytes) beyond %s (%llu bytes)", what, (unsigned long long)elem,
             (unsigned long long)esz, reg->what.c_str(), (unsigned long long)(reg->hi - reg->lo));
}

uint64_t emu_deposit(uint64_t v, const uint8_t *pos, int nbits) {
  uint64_t r = 0;
  for (int i = 0; i < nbits; ++i) r |= ((v >> i) & 1ull) << pos[i];
  return r;
}

int emu_down_opts(int s) { return (s == 1 || s == 2) ? 3 : 2; }
int emu_down_prep(int s, int o) { return (s == 1 || s == 2) ? (o == 0 ? s + 1 : o - 1) : o; }

// transform_elem's enumeration for one entry: returns the number of terms
uint64_t emu_transform_entry(const EmuRegions &R, const TransformArgs &a, uint64_t e) {
  if (a.c < 0 || a.c > kMaxCutsT || a.o < 0 || a.u < 0 || a.o + a.u > 62) emu_fail("transform: c %d o %d u %d", a.c, a.o, a.u);
  const uint64_t cols = 1ull << (a.o + a.u);
  const uint64_t x = e & ((1ull << a.o) - 1);
  const uint64_t row = e >> a.o;
  uint32_t opt = 0;
  uint64_t terms = 0;
  while (true) {
    uint64_t rin = 0, b = 0;
    for (int t = 0; t < a.c; ++t) {
      const int s = (int)((row >> (2 * (a.c - 1 - t))) & 3);
      const int o = (int)((opt >> (2 * t)) & 3u);
      if (a.up[t]) {
        if (a.bbit[t] < 0 || a.bbit[t] >= a.u) emu_fail("transform: measured bit %d of %d", a.bbit[t], a.u);
        rin += (uint64_t)((s == 3) ? 0 : s) * a.w[t];
        b |= (uint64_t)o << a.bbit[t];
      } else {
        rin += (uint64_t)emu_down_prep(s, o) * a.w[t];
      }
    }
    emu_access(R, a.raw, rin * cols + ((x << a.u) | b), 8, "transform read");
    if (++terms > 43046721ull) emu_fail("transform: option loop does not end");
    int t = a.c - 1;
    for (; t >= 0; --t) {
      const int s = (int)((row >> (2 * (a.c - 1 - t))) & 3);
      const uint32_t n = a.up[t] ? 2u : (uint32_t)emu_down_opts(s);
      const uint32_t o = ((opt >> (2 * t)) & 3u) + 1u;
      opt &= ~(3u << (2 * t));
      if (o < n) {
        opt |= o << (2 * t);
        break;
      }
    }
    if (t < 0) break;
  }
  emu_access(R, a.out, e, 8, "transform write");
  return terms;
}

int emu_plane_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

void emu_pack_entry(const EmuRegions &R, const PackArgs &a, uint64_t e) {
  uint64_t src = a.base;
  for (int i = 0; i < a.nbits; ++i) src += ((e >> i) & 1ull) << a.inpos[i];
  emu_access(R, a.src, src, 8, "pack read");
  if (a.dexp) emu_access(R, a.dexp, 0, 4, "pack exponent read");
  const uint64_t kmask = (1ull << a.lk) - 1;
  const uint64_t d = ((e >> a.lk) << a.kpad) | (e & kmask);
  const int eb = emu_plane_bytes(a.prec);
  emu_access(R, a.dst0, d, eb, "pack write (plane 0)");
  if (a.prec >= 2) emu_access(R, a.dst1, d, eb, "pack write (plane 1)");
  if (a.prec >= 3) emu_access(R, a.dst2, d, eb, "pack write (plane 2)");
}

void emu_gemm_tile(const EmuRegions &R, const GemmArgs &g, int prec, int tile, uint64_t t) {
  const int BM = tile_bm(tile), BN = BM;
  int BK = 32;
  if (prec == 0) BK = 16;
  else if (prec == 1) BK = (g.lk > 8 || g.kpad >= 5) ? 32 : 16;
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln, KP = 1ull << g.kpad;
  if (g.ksplit) emu_fail("gemm: split k inside the batch");
  if (KP % BK) emu_fail("gemm: row stride 2^%d is not a multiple of the k step %d", g.kpad, BK);
  const uint64_t tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  if (t >= tilesM * tilesN) emu_fail("gemm: tile %llu of %llu", (unsigned long long)t,
                                     (unsigned long long)(tilesM * tilesN));
  if (g.swz) emu_fail("gemm: swizzled placement inside the batch");
  const uint64_t tm = t / tilesN, tn = t % tilesN;
  const uint64_t m0 = tm * BM, n0 = tn * BN;
  const int planes = prec == 2 ? 2 : (prec == 3 ? 3 : 1);
  const int eb = emu_plane_bytes(prec);
  const void *A[3] = {g.a0, g.a1, g.a2}, *B[3] = {g.b0, g.b1, g.b2};
  for (int p = 0; p < planes; ++p)
    for (uint64_t r = m0; r < std::min(M, m0 + BM); ++r) {
      emu_access(R, A[p], r * KP, eb, "gemm A row start");
      emu_access(R, A[p], r * KP + KP - 1, eb, "gemm A row end");
    }
  for (int p = 0; p < planes; ++p)
    for (uint64_t r = n0; r < std::min(N, n0 + BN); ++r) {
      emu_access(R, B[p], r * KP, eb, "gemm B row start");
      emu_access(R, B[p], r * KP + KP - 1, eb, "gemm B row end");
    }
  if (g.dscale) emu_access(R, g.dscale, 0, 8, "gemm scale read");
  const int oeb = g.out_kind == OUT_F64 || g.out_kind == OUT_F64_ACC ? 8 : (g.out_kind == OUT_F32 ? 4 : 2);
  const int lbm = __builtin_ctz(BM), lbn = __builtin_ctz(BN);
  const bool staged = prec != 0 && g.staged;
  const uint64_t base = emu_deposit(m0, g.posM, g.lm) + emu_deposit(n0, g.posN, g.ln);
  for (uint64_t i = 0; i < (uint64_t)BM && m0 + i < M; ++i)
    for (uint64_t j = 0; j < (uint64_t)BN && n0 + j < N; ++j) {
      const uint64_t addr = emu_deposit(m0 + i, g.posM, g.lm) + emu_deposit(n0 + j, g.posN, g.ln);
      if (staged) {
        const uint64_t x = emu_deposit(i, g.rankM, lbm) | emu_deposit(j, g.rankN, lbn);
        if (x >= (uint64_t)(BM * BN)) emu_fail("gemm: staged index %llu", (unsigned long long)x);
        if (base + emu_deposit(x, g.lpos, g.ncompact) != addr) emu_fail("gemm: staged address differs");
        if (g.vec4 && (addr & 3) != (x & 3)) emu_fail("gemm: float4 run misaligned");
      }
      emu_access(R, g.c0, addr, oeb, "gemm write (plane 0)");
      if (g.out_kind == OUT_SPLIT2 || g.out_kind == OUT_SPLIT3) emu_access(R, g.c1, addr, oeb, "gemm write (plane 1)");
      if (g.out_kind == OUT_SPLIT3) emu_access(R, g.c2, addr, oeb, "gemm write (plane 2)");
    }
}
}  // namespace

static std::string batch_emulate(int njobs, Plan *const *plans, const uint64_t *out_bytes, uint64_t max_terms) {
  if (njobs < 1 || !plans) return "no jobs";
  // swap in synthetic addresses
  struct Saved { Plan *p; void *ws; std::vector<std::pair<double *, double *>> t; };
  std::vector<Saved> saved;
  for (int j = 0; j < njobs; ++j) {
    for (int i = 0; i < j; ++i)
      if (plans[i] == plans[j] || plans[i]->net == plans[j]->net) return "two jobs share a plan or network";
    Saved sv{plans[j], plans[j]->ws, {}};
    for (auto &t : plans[j]->net->t) sv.t.push_back({t.dev_raw, t.dev_pauli});
    saved.push_back(sv);
  }
  EmuRegions R;
  std::vector<void *> outs(njobs);
  std::string err;
  try {
    const int prec = int(plans[0]->prec);
    for (int j = 0; j < njobs; ++j) {
      Plan *p = plans[j];
      if (int(p->prec) != prec || p->prec == Prec::F16X3 || p->num_slices != 1)
        return "jobs must share one precision other than fp16x3 and be unsliced";
      char nm[64];
      for (size_t ti = 0; ti < p->net->t.size(); ++ti) {
        auto &t = p->net->t[ti];
        snprintf(nm, sizeof(nm), "job %d tensor %zu input", j, ti);
        t.dev_raw = (double *)R.fresh(t.rows * t.cols * 8, nm);
      }
      snprintf(nm, sizeof(nm), "job %d workspace", j);
      p->ws = R.fresh(p->ws_bytes, nm);
      uint64_t off = 0;
      for (auto &t : p->net->t) {
        if (t.basis == TQC_BASIS_RAW) {
          t.dev_pauli = (double *)((char *)p->ws + off);
          off = (off + t.pauli_entries() * 8 + 255) & ~uint64_t(255);
        } else {
          t.dev_pauli = t.dev_raw;
        }
      }
      const uint64_t need = (1ull << p->out_bits) * (p->out_dtype == TQC_F64 ? 8 : 4);
      snprintf(nm, sizeof(nm), "job %d output", j);
      outs[j] = R.fresh(out_bytes ? out_bytes[j] : need, nm);
    }
    BatchTables T = build_batch_tables(njobs, plans, outs.data(), prec);
    // finer regions inside each workspace: every node plane and Pauli tensor
    for (int j = 0; j < njobs; ++j) {
      Plan *p = plans[j];
      for (size_t i = 0; i < p->nodes.size(); ++i) {
        const Node &nd = p->nodes[i];
        if (nd.plane_bytes == 0) continue;
        for (int q = 0; q < nd.planes; ++q)
          R.add((char *)p->ws + nd.offset + q * nd.plane_bytes, nd.elems() * emu_plane_bytes(prec == 4 ? 1 : prec),
                "job " + std::to_string(j) + " node " + std::to_string(i) + " plane " + std::to_string(q));
      }
      for (size_t ti = 0; ti < p->net->t.size(); ++ti) {
        const auto &t = p->net->t[ti];
        if (t.basis == TQC_BASIS_RAW)
          R.add(t.dev_pauli, t.pauli_entries() * 8, "job " + std::to_string(j) + " Pauli tensor " + std::to_string(ti));
      }
    }
    unsigned long long *d_max = (unsigned long long *)R.fresh(std::max(1, T.nleaves) * 8, "leaf abs-max bits");
    int *d_exp = (int *)R.fresh(std::max(1, T.nleaves) * 4, "leaf exponents");
    double *d_rs = (double *)R.fresh(njobs * 8, "job scales");
    for (const BatchTables::Fix &f : T.fixes) {
      if (f.kind == 0) T.aargs[f.idx].out = d_max + f.leaf;
      else if (f.kind == 1) T.pargs[f.idx].dexp = d_exp + f.leaf;
      else T.gargs[f.idx].dscale = d_rs + f.job;
    }
    // pre-pass: transform
    uint64_t terms = 0;
    for (const TransformArgs &a : T.targs) {
      const uint64_t n = (1ull << (2 * a.c)) << a.o;
      for (uint64_t e = 0; e < n; ++e) {
        terms += emu_transform_entry(R, a, e);
        if (terms > max_terms) emu_fail("emulation budget exceeded (transform)");
      }
    }
    // pre-pass: abs-max, exponents, scales
    if ((int)T.aargs.size() != T.nleaves) emu_fail("abs-max records %zu for %d leaves", T.aargs.size(), T.nleaves);
    for (const AbsMaxArgs &a : T.aargs) {
      if (a.nbits < 0 || a.nbits > kMaxBits) emu_fail("abs-max: %d bits", a.nbits);
      for (uint64_t e = 0; e < (1ull << a.nbits); ++e) {
        uint64_t src = a.base;
        for (int i = 0; i < a.nbits; ++i) src += ((e >> i) & 1ull) << a.inpos[i];
        emu_access(R, a.src, src, 8, "abs-max read");
      }
      emu_access(R, a.out, 0, 8, "abs-max result");
    }
    if ((int)T.job_leaf0.size() != njobs + 1) emu_fail("leaf offsets");
    for (int j = 0; j < njobs; ++j) {
      if (T.job_leaf0[j] > T.job_leaf0[j + 1] || T.job_leaf0[j + 1] > T.nleaves) emu_fail("leaf range of job %d", j);
      for (int l = T.job_leaf0[j]; l < T.job_leaf0[j + 1]; ++l) {
        emu_access(R, d_max, l, 8, "scale: abs-max read");
        emu_access(R, d_exp, l, 4, "scale: exponent write");
      }
      emu_access(R, d_rs, j, 8, "scale: job scale write");
    }
    // units, levels, items
    const int nunits = (int)T.fin.size();
    std::vector<int> level_of(nunits, -1);
    for (size_t L = 0; L + 1 < T.level_first.size(); ++L)
      for (int u = 0; u < nunits; ++u)
        if (T.fin[u].first >= T.level_first[L] && T.fin[u].first < T.level_first[L + 1]) level_of[u] = (int)L;
    for (int u = 0; u < nunits; ++u) {
      const BatchUnit &bu = T.fin[u];
      if (level_of[u] < 0) emu_fail("unit %d in no level", u);
      if (bu.ntiles == 0 || bu.ntiles >= (1ull << 32)) emu_fail("unit %d: %llu items", u, (unsigned long long)bu.ntiles);
      if (bu.first + bu.ntiles > T.level_first[level_of[u] + 1]) emu_fail("unit %d crosses a level", u);
      for (int d : {bu.dep0, bu.dep1})
        if (d >= 0 && (d >= u || level_of[d] >= level_of[u])) emu_fail("unit %d depends on unit %d of a later level", u, d);
      if (bu.kind == UNIT_PACK) {
        if (bu.arg < 0 || bu.arg >= (int)T.pargs.size()) emu_fail("unit %d: pack record %d", u, bu.arg);
      } else if (bu.kind == UNIT_GEMM) {
        if (bu.arg < 0 || bu.arg >= (int)T.gargs.size()) emu_fail("unit %d: gemm record %d", u, bu.arg);
        if (bu.tile < 0 || bu.tile > 2) emu_fail("unit %d: tile %d", u, bu.tile);
      } else {
        emu_fail("unit %d: kind %d", u, bu.kind);
      }
    }
    for (uint64_t item = 0; item < T.total; ++item) {
      int lo = 0, hi = nunits - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T.fin[mid].first <= item) lo = mid;
        else hi = mid - 1;
      }
      const BatchUnit &bu = T.fin[lo];
      if (item < bu.first || item >= bu.first + bu.ntiles) emu_fail("item %llu maps to unit %d", (unsigned long long)item, lo);
      const uint64_t t = item - bu.first;
      if (bu.kind == UNIT_PACK) {
        const PackArgs &a = T.pargs[bu.arg];
        const uint64_t total = 1ull << a.nbits;
        const uint64_t e1 = std::min(total, (t + 1) * 4096);
        for (uint64_t e = t * 4096; e < e1; ++e) emu_pack_entry(R, a, e);
      } else {
        emu_gemm_tile(R, T.gargs[bu.arg], prec, bu.tile, t);
      }
    }
  } catch (const EmuFail &f) {
    err = f.msg;
  } catch (const Error &e) {
    err = e.msg;
  }
  for (const Saved &sv : saved) {
    sv.p->ws = sv.ws;
    for (size_t i = 0; i < sv.t.size(); ++i) {
      sv.p->net->t[i].dev_raw = sv.t[i].first;
      sv.p->net->t[i].dev_pauli = sv.t[i].second;
    }
  }
  return err;
}

// --------------------------------------------------------------- autotune
// Measured tile choice per step shape (precision, log2 M, N, K); the table
// is process-wide and can be saved to / loaded from a text file.
struct TuneKey {
  int prec, lm, ln, lk;
  bool operator<(const TuneKey &o) const {
    return std::tie(prec, lm, ln, lk) < std::tie(o.prec, o.lm, o.ln, o.lk);
  }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<int, double>> g_tune;

static void apply_tuned_tiles(Plan *p) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (Step &st : p->steps) {
    auto it = g_tune.find(TuneKey{int(p->prec), st.lm, st.ln, st.lk});
    if (it != g_tune.end()) st.tile = it->second.first;
  }
}

static void autotune_plan(Plan *p, void *out, uint64_t out_bytes, int reps, hipStream_t s) {
  if (p->num_slices != 1) fail(TQC_ERR_UNSUPPORTED, "autotuning needs an unsliced plan");
  execute(p, out, out_bytes, s);  // valid operands for every step
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int root_kind = p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32;
  const ScaleBuf sb = scale_buffers(p);
  for (Step &st : p->steps) {
    GemmArgs g = make_gemm_args(p, st, out, root_kind, sb.root_scale);
    int best = st.tile;
    double best_ms = 1e30;
    for (int tile = 0; tile < 3; ++tile) {
      const int bm = tile_bm(tile);
      if (tile != 2 && (st.lm < 5 || st.ln < 5) && bm > 32) continue;
      // time the step as execute runs it: a final step with tile 0 that
      // qualifies runs on the persistent final-step kernel
      Step trial = st;
      trial.tile = tile;
      const int sp = step_prec(p, st);
      const bool persistent = root_on_persistent(p, trial, g);
      auto run = [&]() {
        if (persistent) HIP_OK(launch_root_gemm(sp, g, s));
        else HIP_OK(launch_gemm(sp, g, tile, s, p->tile_policy == 2));
      };
      run();  // warm
      HIP_OK(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) run();
      HIP_OK(hipEventRecord(e1, s));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / reps;
      if (per < best_ms) {
        best_ms = per;
        best = tile;
      }
    }
    st.tile = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{int(p->prec), st.lm, st.ln, st.lk}] = {best, best_ms};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}


// ------------------------------------------------- heavy state selection
// Sec. IV, Alg. 1: per tensor, the L2 norm of every output state over all
// edge permutations (rows of the Pauli-basis tensor), computed on the device
// in float64; then on the host every tensor starts with its heaviest state
// and the other states join in descending norm order (ties: smaller tensor,
// then smaller state) while the product of the subset sizes is below s_max.
struct DevMem {
  void *p = nullptr;
  explicit DevMem(size_t bytes) { HIP_OK(hipMalloc(&p, bytes ? bytes : 8)); }
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
};

// device Pauli tensor of tensor j: the resident one, or transformed into `tmp`
static const double *pauli_on_device(const TensorIn &t, std::unique_ptr<DevMem> &tmp, hipStream_t s) {
  if (t.basis == TQC_BASIS_PAULI) return t.dev_raw;
  tmp.reset(new DevMem(t.pauli_entries() * 8));
  transform_tensor(t, (double *)tmp->p, s);
  return (const double *)tmp->p;
}

static void hss_norms(Network *net, std::vector<std::vector<double>> &norms, hipStream_t s) {
  upload(net);
  check_device(net->device);
  norms.assign(net->m, {});
  for (int j = 0; j < net->m; ++j) {
    const TensorIn &t = net->t[j];
    const uint64_t rows = 1ull << (2 * t.cuts.size()), cols = 1ull << t.outputs.size();
    std::unique_ptr<DevMem> tmp;
    const double *src = pauli_on_device(t, tmp, s);
    DevMem partial(colnorm_scratch_entries(rows, cols) * 8), dn(cols * 8);
    HIP_OK(launch_column_norms(src, rows, cols, (double *)partial.p, (double *)dn.p, s));
    norms[j].resize(cols);
    HIP_OK(hipMemcpyAsync(norms[j].data(), dn.p, cols * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
}

static std::vector<std::vector<int32_t>> hss_choose(const std::vector<std::vector<double>> &norms,
                                                    uint64_t s_max) {
  struct Cand {
    double v;
    int j;
    int32_t i;
  };
  const int m = (int)norms.size();
  std::vector<std::vector<int32_t>> sel(m);
  std::vector<Cand> rest;
  for (int j = 0; j < m; ++j) {
    int32_t first = 0;
    for (int32_t i = 1; i < (int32_t)norms[j].size(); ++i)
      if (norms[j][i] > norms[j][first]) first = i;
    sel[j].push_back(first);
    for (int32_t i = 0; i < (int32_t)norms[j].size(); ++i)
      if (i != first) rest.push_back({norms[j][i], j, i});
  }
  std::sort(rest.begin(), rest.end(), [](const Cand &a, const Cand &b) {
    if (a.v != b.v) return a.v > b.v;
    if (a.j != b.j) return a.j < b.j;
    return a.i < b.i;
  });
  unsigned __int128 size = 1;  // stays below 2 * s_max <= 2^65
  for (size_t pos = 0; size < s_max && pos < rest.size(); ++pos) {
    const Cand &c = rest[pos];
    const uint64_t k = sel[c.j].size();
    size = size / k * (k + 1);
    sel[c.j].push_back(c.i);
  }
  for (auto &v : sel) std::sort(v.begin(), v.end());
  return sel;
}

static int ceil_log2(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) ++b;
  return b;
}

// The network restricted to chosen output states: tensor j keeps the
// columns states_j (ascending), padded with zero columns to 2^b_j, b_j =
// ceil(log2 |states_j|); its b_j output qubits are numbered after those of
// tensors 0..j-1.  Contracting it gives P at every retained product state
// (entry sum_j y_j 2^off_j holds the state whose tensor-j bits are
// states_j[y_j]); entries with a padding index are exactly zero.
static Network *select_states_network(Network *src, const int32_t *counts, const int32_t *states, hipStream_t s) {
  upload(src);
  check_device(src->device);
  const int m = src->m;
  std::unique_ptr<Network> net(new Network());
  net->m = m;
  net->K = src->K;
  net->cuts = src->cuts;
  net->t.resize(m);
  int nq = 0;
  uint64_t at = 0;
  for (int j = 0; j < m; ++j) {
    const TensorIn &t = src->t[j];
    const uint64_t cols = 1ull << t.outputs.size();
    const int32_t cnt = counts[j];
    if (cnt < 1 || (uint64_t)cnt > cols) fail(TQC_ERR_INVALID_ARG, "tensor %d: %d states of %llu", j, cnt,
                                              (unsigned long long)cols);
    for (int32_t y = 0; y < cnt; ++y) {
      const int32_t v = states[at + y];
      if (v < 0 || (uint64_t)v >= cols || (y > 0 && v <= states[at + y - 1]))
        fail(TQC_ERR_INVALID_ARG, "tensor %d: states must be ascending and below %llu", j, (unsigned long long)cols);
    }
    TensorIn &d = net->t[j];
    d.cuts = t.cuts;
    d.up = t.up;
    d.u = t.u;
    d.d = t.d;
    d.basis = TQC_BASIS_PAULI;
    const int b = ceil_log2((uint64_t)cnt);
    for (int i = 0; i < b; ++i) d.outputs.push_back(nq + i);
    nq += b;
    d.rows = 1ull << (2 * t.cuts.size());
    d.cols = 1ull << b;
    HIP_OK(hipMalloc((void **)&d.dev_raw, d.rows * d.cols * 8));
    d.dev_pauli = d.dev_raw;
    std::unique_ptr<DevMem> tmp;
    const double *pt = pauli_on_device(t, tmp, s);
    DevMem dstates((size_t)cnt * 4);
    HIP_OK(hipMemcpyAsync(dstates.p, states + at, (size_t)cnt * 4, hipMemcpyHostToDevice, s));
    HIP_OK(launch_gather_columns(pt, d.rows, cols, (const int32_t *)dstates.p, (uint64_t)cnt, d.cols, d.dev_raw, s));
    HIP_OK(hipStreamSynchronize(s));
    at += cnt;
  }
  net->n = nq;
  net->device = src->device;
  net->uploaded = true;
  return net.release();
}

// ------------------------------------------------------------- multi-job
// Many independent reconstructions as one HIP graph: every job's plain
// launches (transform, packs, pairwise steps, final step) are captured once,
// spread over a few streams (largest predicted jobs first, each to the
// least-loaded stream), and the graph is replayed per call.  Independent
// branches let the device run small jobs side by side and the replay costs
// one launch instead of a few per job.  Every allocation happens at creation,
// outside the capture.  With `timed`, one-thread kernels store the device
// clock before and after every job (kernels rather than timing events, so the
// stamps are ordinary graph nodes).
struct Multi {
  std::vector<Plan *> plans;
  std::vector<void *> outs;
  std::vector<uint64_t> out_bytes;
  std::vector<int> stream_of;     // job -> worker stream
  std::vector<int> order;         // launch order (largest first)
  int device = -1;
  bool use_graph = true, timed = false;
  double tick_ms = 0.0;           // milliseconds per clock tick
  unsigned long long *stamps = nullptr;  // [0] = launch, [1 + 2j] / [2 + 2j] = job j start / end
  std::vector<hipStream_t> streams;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join, mid;
  hipStream_t last_stream = nullptr;
  bool ran = false;
  // grouped mode: the work of all jobs as a short list of shared launches
  // (built at creation, replayed by each execute); stamp slot of each step
  // and, per job, the step that completes it
  bool grouped = false;
  // grouped heads: only the launches before the pairwise steps are shared
  // (one list per wave on the last stream); every job then runs its own
  // pairwise steps and final step on its worker stream
  bool heads_only = false;
  std::vector<std::vector<int>> wave_jobs;  // jobs of each wave, largest first
  struct Wave {
    std::vector<std::function<void(hipStream_t)>> steps;  // up to the final steps
    std::vector<std::function<void(hipStream_t)>> roots;  // shared persistent final steps
  };
  std::vector<Wave> waves;
  std::vector<hipEvent_t> head_done;  // per wave: its steps are done
  std::vector<int> done_at;       // job -> stamp slot of the launch that completes it
  int nslots = 0;                 // stamp slots in use
  int shared_roots = 0;           // persistent final-step launches
  int shared_root_jobs = 0;       // jobs whose final step runs in one of them
  void *gtab = nullptr;           // device tables of the grouped launches
  ~Multi() {
    if (gtab) (void)hipFree(gtab);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : join) (void)hipEventDestroy(e);
    for (auto e : mid) (void)hipEventDestroy(e);
    for (auto e : head_done) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto st : streams) (void)hipStreamDestroy(st);
    if (cap) (void)hipStreamDestroy(cap);
    if (stamps) (void)hipFree(stamps);
  }
};

// ----------------------------------------------------------- grouped mode
// The launches one single-slice execute makes (run_slices), as records:
// transform passes by pass level, per-entry transforms, the operand scales
// (zero, abs-max, exponents), the leaf packs, and the pairwise steps with
// their depth in the contraction tree (1 + the deeper operand's depth).
struct JobOps {
  std::vector<std::vector<TransformPassArgs>> pass_levels;
  std::vector<TransformArgs> transforms;
  bool scaled = false;  // m >= 2: zero / abs-max / exponents
  ZeroRec zero{};
  std::vector<AbsMaxArgs> absmax;  // leaves whose abs-max no transform takes
  ScaleRec scale{};
  std::vector<PackArgs> packs;
  struct GemmOp {
    GemmArgs g;
    int sp, tile, depth;
    bool root, persistent;
  };
  std::vector<GemmOp> gemms;
  // float16-split plans: the split of the final step's operands
  bool f16 = false;
  const float *f16_src[2] = {nullptr, nullptr};
  uint64_t f16_n[2] = {0, 0};
  uint16_t *f16_hi[2] = {nullptr, nullptr}, *f16_lo[2] = {nullptr, nullptr};
  unsigned long long *f16_max = nullptr;
  const double *f16_rs = nullptr;
  double *f16_rs2 = nullptr;
};

static JobOps job_ops(Plan *p, void *out) {
  JobOps o;
  Network &net = *p->net;
  const int m = net.m;
  const int root_kind = p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32;
  // as in a plan's own execution: the transforms take the abs-max of the
  // leaves they write, the others get abs-max records
  const bool scaled = m >= 2;
  ScaleBuf sb{};
  if (scaled) sb = scale_buffers(p);
  for (int j = 0; j < m; ++j) {
    TensorIn &t = net.t[j];
    const AbsMaxOut am = scaled ? fused_absmax(p, sb, j) : AbsMaxOut{};
    if (scaled && !am.p) o.absmax.push_back(absmax_record(p, sb, j));
    if (t.basis != TQC_BASIS_RAW) continue;
    if ((int)t.cuts.size() >= kPassMinCuts) {
      char *b = (char *)p->ws + p->tscr_off[j];
      schedule_passes(t, t.dev_pauli, (double *)b, (double *)(b + p->tscr_bytes[j]), p->tscr_bytes[j], o.pass_levels,
                      am);
    } else {
      TransformArgs a = make_transform_args(t, t.dev_pauli);
      a.amax = am.p;
      a.amask = am.mask;
      a.abase = am.base;
      o.transforms.push_back(a);
    }
  }
  if (m == 1) {
    o.packs.push_back(make_pack_args(p, 0, out, nullptr, nullptr, root_kind == OUT_F64 ? 0 : 1, 0));
    return o;
  }
  o.scaled = true;
  o.zero = ZeroRec{sb.maxbits, (uint64_t)m};
  o.scale = ScaleRec{sb.maxbits, m, net.K, sb.exps, sb.root_scale};
  for (int j = 0; j < m; ++j) {
    Node &nd = p->nodes[j];
    char *b = (char *)p->ws + nd.offset;
    o.packs.push_back(make_pack_args(p, j, b, nd.planes > 1 ? b + nd.plane_bytes : nullptr,
                                     nd.planes > 2 ? b + 2 * nd.plane_bytes : nullptr, pack_prec(p), 0, sb.exps + j));
  }
  std::vector<int> depth(p->nodes.size(), 0);
  for (const Step &st : p->steps) {
    depth[st.out] = 1 + std::max(depth[st.a], depth[st.b]);
    JobOps::GemmOp op;
    op.g = make_gemm_args(p, st, out, root_kind, sb.root_scale);
    op.sp = step_prec(p, st);
    op.tile = st.tile;
    op.depth = depth[st.out];
    op.root = st.root;
    op.persistent = root_on_persistent(p, st, op.g);
    if (st.root && p->prec == Prec::F16X3) {
      const Node &na = p->nodes[st.a], &nb = p->nodes[st.b];
      char *ha = (char *)p->ws + p->h16_off[0], *hb = (char *)p->ws + p->h16_off[1];
      o.f16 = true;
      o.f16_src[0] = (const float *)((char *)p->ws + na.offset);
      o.f16_src[1] = (const float *)((char *)p->ws + nb.offset);
      o.f16_n[0] = na.elems();
      o.f16_n[1] = nb.elems();
      o.f16_hi[0] = (uint16_t *)ha;
      o.f16_lo[0] = (uint16_t *)(ha + p->h16_plane[0]);
      o.f16_hi[1] = (uint16_t *)hb;
      o.f16_lo[1] = (uint16_t *)(hb + p->h16_plane[1]);
      o.f16_max = sb.maxbits16;
      o.f16_rs = sb.root_scale;
      o.f16_rs2 = sb.root_scale2;
    }
    o.gemms.push_back(op);
  }
  return o;
}

// Device tables of the grouped launches, laid out in one allocation.
struct TableArena {
  std::vector<unsigned char> host;
  uint64_t add(const void *p, uint64_t bytes) {
    const uint64_t off = (host.size() + 255) & ~uint64_t(255);
    host.resize(off + bytes);
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <typename T>
  uint64_t add_vec(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

// A grouped launch over records of one kind: the records' own workgroup
// counts become the first-workgroup offsets.
template <typename T>
struct Group {
  std::vector<T> recs;
  std::vector<uint32_t> first{0};
  void push(const T &r, uint32_t blocks) {
    recs.push_back(r);
    const uint64_t next = (uint64_t)first.back() + blocks;
    if (next > 0x7fffffffull) fail(TQC_ERR_UNSUPPORTED, "grouped launch of more than 2^31 workgroups");
    first.push_back((uint32_t)next);
  }
  bool empty() const { return recs.empty(); }
};

// The whole batch as a short list of launches on one stream: pass levels,
// per-entry transforms, scales (zero, abs-max, exponents), packs, then the
// pairwise steps depth by depth (one launch per kernel variant and depth;
// steps the plain launcher would split over k run alone, with that split;
// float16 splits before their final step), and last the final steps that run
// on the persistent kernel, one launch per (form, K).  Every record is the
// one the job's own execute would launch, so outputs match bit for bit.
using LaunchFactory = std::function<std::function<void(hipStream_t)>(char *)>;

struct WavePlan {
  std::vector<LaunchFactory> steps, roots;
  std::vector<std::vector<int>> step_jobs, root_jobs;  // jobs each launch completes
};

// The launches of one wave (a subset of the jobs, `sel`), their tables in A.
static WavePlan plan_wave(Multi *b, const std::vector<int> &sel, std::vector<JobOps> &all_ops, TableArena &A,
                          bool heads_only) {
  WavePlan W;
  const int njobs = (int)sel.size();
  std::vector<JobOps> ops(njobs);
  for (int q = 0; q < njobs; ++q) ops[q] = all_ops[sel[q]];
  auto add_launch = [&](LaunchFactory f, std::vector<int> jobs = {}) {
    for (int &x : jobs) x = sel[x];
    W.steps.push_back(std::move(f));
    W.step_jobs.push_back(std::move(jobs));
  };
  // 0. the abs-max accumulators start from zero (the transforms take maxima)
  {
    std::vector<ZeroRec> zr;
    for (auto &o : ops)
      if (o.scaled) zr.push_back(o.zero);
    if (!zr.empty()) {
      const uint64_t zo = A.add_vec(zr);
      const int nz = (int)zr.size();
      add_launch([=](char *d) {
        return [=](hipStream_t s) { HIP_OK(launch_grouped_zero((const ZeroRec *)(d + zo), nz, s)); };
      });
    }
  }
  // 1. transform passes, level by level, then per-entry transforms
  size_t nlev = 0;
  for (auto &o : ops) nlev = std::max(nlev, o.pass_levels.size());
  for (size_t L = 0; L < nlev; ++L) {
    Group<TransformPassArgs> g;
    for (auto &o : ops)
      if (L < o.pass_levels.size())
        for (auto &a : o.pass_levels[L]) {
          if (a.nseg < 1 || a.nseg > kPassSegs || a.g < 1 || a.g > 2) fail(TQC_ERR_INTERNAL, "transform pass record");
          g.push(a, grouped_pass_blocks(a));
        }
    if (g.empty()) continue;
    const uint64_t ro = A.add_vec(g.recs), fo = A.add_vec(g.first);
    const int n = (int)g.recs.size();
    const uint32_t blocks = g.first.back();
    add_launch([=](char *d) {
      return [=](hipStream_t s) {
        HIP_OK(launch_grouped_passes((const TransformPassArgs *)(d + ro), (const uint32_t *)(d + fo), n, blocks, s));
      };
    });
  }
  {
    Group<TransformArgs> g;
    for (auto &o : ops)
      for (auto &a : o.transforms) g.push(a, grouped_transform_blocks(a));
    if (!g.empty()) {
      const uint64_t ro = A.add_vec(g.recs), fo = A.add_vec(g.first);
      const int n = (int)g.recs.size();
      const uint32_t blocks = g.first.back();
      add_launch([=](char *d) {
        return [=](hipStream_t s) {
          HIP_OK(launch_grouped_transforms((const TransformArgs *)(d + ro), (const uint32_t *)(d + fo), n, blocks, s));
        };
      });
    }
  }
  // 2. scales: abs-max of leaves no transform wrote, then exponents
  {
    std::vector<ScaleRec> sr;
    Group<AbsMaxArgs> g;
    for (auto &o : ops) {
      if (!o.scaled) continue;
      sr.push_back(o.scale);
      for (auto &a : o.absmax) g.push(a, grouped_absmax_blocks(a));
    }
    if (!g.empty()) {
      const uint64_t ro = A.add_vec(g.recs), fo = A.add_vec(g.first);
      const int n = (int)g.recs.size();
      const uint32_t blocks = g.first.back();
      add_launch([=](char *d) {
        return [=](hipStream_t s) {
          HIP_OK(launch_grouped_absmax((const AbsMaxArgs *)(d + ro), (const uint32_t *)(d + fo), n, blocks, s));
        };
      });
    }
    if (!sr.empty()) {
      const uint64_t so = A.add_vec(sr);
      const int nz = (int)sr.size();
      add_launch([=](char *d) {
        return [=](hipStream_t s) { HIP_OK(launch_grouped_scales((const ScaleRec *)(d + so), nz, s)); };
      });
    }
  }
  // 3. packs (a single-tensor job's pack is its whole result)
  {
    Group<PackArgs> g;
    std::vector<int> done;
    for (int j = 0; j < njobs; ++j) {
      for (auto &a : ops[j].packs) g.push(a, grouped_pack_blocks(a));
      if (b->plans[sel[j]]->net->m == 1) done.push_back(j);
    }
    if (!g.empty()) {
      const uint64_t ro = A.add_vec(g.recs), fo = A.add_vec(g.first);
      const int n = (int)g.recs.size();
      const uint32_t blocks = g.first.back();
      add_launch([=](char *d) {
        return [=](hipStream_t s) {
          HIP_OK(launch_grouped_packs((const PackArgs *)(d + ro), (const uint32_t *)(d + fo), n, blocks, s));
        };
      }, done);
    }
  }
  if (heads_only) return W;
  // 4. pairwise steps by depth; persistent final steps collected for the end
  int maxd = 0;
  for (auto &o : ops)
    for (auto &op : o.gemms) maxd = std::max(maxd, op.depth);
  std::map<std::pair<int, int>, std::vector<std::pair<int, RootJob>>> roots;
  for (int dpt = 1; dpt <= maxd; ++dpt) {
    // float16 splits of final steps at this depth come first
    for (int j = 0; j < njobs; ++j) {
      const JobOps &o = ops[j];
      if (!o.f16) continue;
      bool here = false;
      for (auto &op : o.gemms) here |= op.root && op.depth == dpt;
      if (!here) continue;
      add_launch([o](char *) {
        return [o](hipStream_t s) {
          HIP_OK(launch_f16_split(o.f16_src[0], o.f16_n[0], o.f16_hi[0], o.f16_lo[0], o.f16_src[1], o.f16_n[1],
                                  o.f16_hi[1], o.f16_lo[1], o.f16_max, o.f16_rs, o.f16_rs2, s));
        };
      });
    }
    std::map<GemmClass, std::pair<Group<GemmArgs>, std::vector<int>>> classes;
    for (int j = 0; j < njobs; ++j)
      for (auto &op : ops[j].gemms) {
        if (op.depth != dpt) continue;
        if (op.persistent) {
          roots[{op.sp, op.g.kpad}].push_back({j, make_root_job(op.sp, op.g)});
          continue;
        }
        const GemmClass c = gemm_class(op.sp, op.g, op.tile);
        if (c.ksplit) {
          // split over k as in the job's own launch (float64 partials in its
          // workspace), so this step runs alone
          const GemmArgs g = op.g;
          const int sp = op.sp, tile = op.tile;
          add_launch([=](char *) {
            return [=](hipStream_t s) { HIP_OK(launch_gemm(sp, g, tile, s)); };
          }, op.root ? std::vector<int>{j} : std::vector<int>{});
          continue;
        }
        GemmArgs g = op.g;
        const int bm = tile_bm(op.tile);
        prepare_gemm_args(g, op.sp, bm, bm);
        g.ksplit = 0;
        if (c.tiles > 0x7fffffffull) fail(TQC_ERR_UNSUPPORTED, "step of more than 2^31 tiles");
        auto &slot = classes[c];
        slot.first.push(g, (uint32_t)c.tiles);
        if (op.root) slot.second.push_back(j);
      }
    for (auto &kv : classes) {
      const GemmClass c = kv.first;
      const Group<GemmArgs> &g = kv.second.first;
      const uint64_t ro = A.add_vec(g.recs), fo = A.add_vec(g.first);
      const int n = (int)g.recs.size();
      const uint32_t blocks = g.first.back();
      add_launch([=](char *d) {
        return [=](hipStream_t s) {
          HIP_OK(launch_grouped_gemm(c, (const GemmArgs *)(d + ro), (const uint32_t *)(d + fo), n, blocks, s));
        };
      }, kv.second.second);
    }
  }
  // 5. final steps on the persistent kernel: one launch per (form, kpad),
  // jobs with the most tiles first (their workgroups start first); per job
  // enough workgroups that the largest job's share per workgroup stays below
  // twice the launch's share per compute unit
  const int cus = std::max(1, root_gemm_warm());
  for (auto &kv : roots) {
    auto &v = kv.second;
    std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.second.ntiles > y.second.ntiles; });
    uint64_t total = 0, most = 0;
    std::vector<RootJob> tab;
    std::vector<int> jobs;
    for (auto &x : v) {
      total += x.second.ntiles;
      most = std::max<uint64_t>(most, x.second.ntiles);
      tab.push_back(x.second);
      jobs.push_back(x.first);
    }
    uint64_t want = (2 * (uint64_t)cus * most + total - 1) / std::max<uint64_t>(total, 1);
    want = std::min<uint64_t>(std::max<uint64_t>(want, 8), (uint64_t)cus);
    const int blocks = (int)((want + 7) & ~7ull);
    const int prec = kv.first.first, kpad = kv.first.second, n = (int)tab.size();
    if (n > 65535) fail(TQC_ERR_UNSUPPORTED, "more than 65535 final steps in one launch");
    const uint64_t ro = A.add_vec(tab);
    W.roots.push_back([=](char *d) {
      return [=](hipStream_t s) { HIP_OK(launch_root_multi(prec, kpad, (const RootJob *)(d + ro), n, blocks, s)); };
    });
    for (int &x : jobs) x = sel[x];
    W.root_jobs.push_back(jobs);
    b->shared_roots += 1;
    b->shared_root_jobs += n;
  }
  return W;
}

// The whole batch as a few waves of jobs (about equal predicted cost each,
// largest jobs first); each wave is a short list of shared launches on its
// own stream, and wave w + 1 starts once wave w's launches before its final
// steps are done, so one wave's final steps (store bound) run beside the
// next wave's earlier launches.
static void build_grouped(Multi *b, int nwaves, bool heads_only) {
  b->grouped = true;
  b->heads_only = heads_only;
  const int njobs = (int)b->plans.size();
  std::vector<JobOps> ops(njobs);
  for (int j = 0; j < njobs; ++j) {
    if (b->plans[j]->num_slices != 1) fail(TQC_ERR_UNSUPPORTED, "job %d: sliced plans are not grouped", j);
    // points the network's Pauli tensors into this plan's workspace (jobs
    // may share a network); the workspace itself exists already
    ensure_workspace(b->plans[j], nullptr);
    ops[j] = job_ops(b->plans[j], b->outs[j]);
  }
  nwaves = std::max(1, std::min(nwaves, njobs));
  std::vector<std::vector<int>> sel(nwaves);
  std::vector<double> load(nwaves, 0.0);
  for (int j : b->order) {
    const int w = int(std::min_element(load.begin(), load.end()) - load.begin());
    sel[w].push_back(j);
    load[w] += std::max(1e-9, b->plans[j]->stats.predicted_seconds);
  }
  TableArena A;
  std::vector<WavePlan> plans;
  for (int w = 0; w < nwaves; ++w)
    if (!sel[w].empty()) {
      plans.push_back(plan_wave(b, sel[w], ops, A, heads_only));
      b->wave_jobs.push_back(sel[w]);
    }
  // upload the tables, then bind the launches to them
  if (!A.host.empty()) {
    HIP_OK(hipMalloc(&b->gtab, A.host.size()));
    HIP_OK(hipMemcpy(b->gtab, A.host.data(), A.host.size(), hipMemcpyHostToDevice));
  }
  b->done_at.assign(njobs, -1);
  int slot = 1 + 2 * njobs;
  for (WavePlan &P : plans) {
    Multi::Wave W;
    for (size_t i = 0; i < P.steps.size(); ++i, ++slot) {
      W.steps.push_back(P.steps[i]((char *)b->gtab));
      for (int j : P.step_jobs[i]) b->done_at[j] = slot;
    }
    for (size_t i = 0; i < P.roots.size(); ++i, ++slot) {
      W.roots.push_back(P.roots[i]((char *)b->gtab));
      for (int j : P.root_jobs[i]) b->done_at[j] = slot;
    }
    b->waves.push_back(std::move(W));
  }
  b->nslots = slot;
  for (int j = 0; j < njobs; ++j)
    if (b->done_at[j] < 0 && !(heads_only && b->plans[j]->net->m >= 2))
      fail(TQC_ERR_INTERNAL, "job %d has no completing launch", j);
}

static Multi *create_multi(int njobs, Plan *const *plans, void *const *outs, const uint64_t *out_bytes,
                           int use_graph, int nstreams, int timed, hipStream_t s, int grouped = 0,
                           int waves = 1) {
  if (njobs < 1 || !plans || !outs) fail(TQC_ERR_INVALID_ARG, "no jobs");
  if (nstreams < 0 || nstreams > 16) fail(TQC_ERR_INVALID_ARG, "streams %d (0..16)", nstreams);
  if (grouped < 0 || grouped > 2) fail(TQC_ERR_INVALID_ARG, "grouped %d (0..2)", grouped);
  if (nstreams == 0) nstreams = 4;
  std::unique_ptr<Multi> b(new Multi());
  b->use_graph = use_graph != 0;
  b->timed = timed != 0;
  HIP_OK(hipGetDevice(&b->device));
  std::vector<double> cost(njobs);
  for (int j = 0; j < njobs; ++j) {
    Plan *p = plans[j];
    if (!p || !outs[j]) fail(TQC_ERR_INVALID_ARG, "job %d: null plan or output", j);
    if (p->num_slices != 1) fail(TQC_ERR_UNSUPPORTED, "job %d: sliced plans are not batched", j);
    if (p->net->device >= 0 && p->net->device != b->device)
      fail(TQC_ERR_DEVICE, "job %d: network lives on device %d, current device is %d", j, p->net->device,
           b->device);
    const uint64_t need = (1ull << p->out_bits) * (p->out_dtype == TQC_F64 ? 8 : 4);
    if (out_bytes && out_bytes[j] < need) fail(TQC_ERR_SHAPE, "job %d: output too small", j);
    // every lazy allocation of the execute path, before any capture
    ensure_workspace(p, s);
    if (p->net->m >= 2) (void)scale_buffers(p);
    b->plans.push_back(p);
    b->outs.push_back(outs[j]);
    b->out_bytes.push_back(need);
    cost[j] = p->stats.predicted_seconds;
  }
  for (int j = 1; j < njobs; ++j)
    for (int i = 0; i < j; ++i)
      if (plans[i] == plans[j]) fail(TQC_ERR_INVALID_ARG, "jobs %d and %d share a plan (and its workspace)", i, j);
  (void)root_gemm_warm();
  b->order.resize(njobs);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<double> load(nstreams, 0.0);
  b->stream_of.assign(njobs, 0);
  for (int j : b->order) {
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    b->stream_of[j] = k;
    load[k] += cost[j];
  }
  if (grouped == 1) {
    build_grouped(b.get(), waves, false);
    nstreams = std::max<int>(nstreams, (int)b->waves.size());
  } else if (grouped == 2) {
    build_grouped(b.get(), waves, true);
    // worker streams by wave: the jobs of each wave, largest first, each to
    // the least-loaded stream; the extra last stream runs the shared launches
    std::fill(load.begin(), load.end(), 0.0);
    for (const auto &wj : b->wave_jobs)
      for (int j : wj) {
        const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
        b->stream_of[j] = k;
        load[k] += cost[j];
      }
    nstreams += 1;
  }
  if (b->timed) {
    int khz = 0;
    HIP_OK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    if (khz <= 0) fail(TQC_ERR_DEVICE, "device reports no clock rate for timestamps");
    b->tick_ms = 1.0 / khz;
    const uint64_t nst = std::max<uint64_t>(1 + 2 * (uint64_t)njobs, (uint64_t)b->nslots);
    HIP_OK(hipMalloc((void **)&b->stamps, nst * 8));
    HIP_OK(launch_zero_u64(b->stamps, nst, s));
  }
  HIP_OK(hipStreamSynchronize(s));
  b->streams.resize(nstreams);
  for (auto &st : b->streams) HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HIP_OK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  HIP_OK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  b->join.resize(nstreams);
  for (auto &e : b->join) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  b->mid.resize(nstreams);
  for (auto &e : b->mid) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  b->head_done.resize(b->waves.size());
  for (auto &e : b->head_done) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return b.release();
}

// A single-slice plan's launches after its leaf packs (pairwise steps, the
// final step), as its execute runs them.
static void run_tail(Plan *p, void *out, hipStream_t s) {
  const ScaleBuf sb = scale_buffers(p);
  run_steps(p, out, p->out_dtype == TQC_F64 ? OUT_F64 : OUT_F32, sb, true, false, s, nullptr, nullptr, nullptr,
            false);
}

// fork from `origin`, every job on its stream (between its two stamps), join
static void multi_enqueue(Multi *b, hipStream_t origin) {
  if (b->timed) HIP_OK(launch_stamp(b->stamps, origin));
  if (b->heads_only) {
    // the waves' shared launches one after another on the last stream; each
    // job's own launches on its worker stream once its wave's are done (a
    // single-tensor job is done with its wave's pack launch: its stamps go
    // around the wave's shared launches)
    hipStream_t hs = b->streams.back();
    const size_t nw = b->streams.size() - 1;
    HIP_OK(hipEventRecord(b->fork, origin));
    for (auto st : b->streams) HIP_OK(hipStreamWaitEvent(st, b->fork, 0));
    for (size_t w = 0; w < b->waves.size(); ++w) {
      if (b->timed)
        for (int j : b->wave_jobs[w])
          if (b->plans[j]->net->m < 2) HIP_OK(launch_stamp(b->stamps + 1 + 2 * j, hs));
      for (auto &f : b->waves[w].steps) f(hs);
      HIP_OK(hipEventRecord(b->head_done[w], hs));
      if (b->timed)
        for (int j : b->wave_jobs[w])
          if (b->plans[j]->net->m < 2) HIP_OK(launch_stamp(b->stamps + 2 + 2 * j, hs));
    }
    for (size_t w = 0; w < b->waves.size(); ++w) {
      std::vector<char> waited(nw, 0);
      for (int j : b->wave_jobs[w]) {
        if (b->plans[j]->net->m < 2) continue;
        const int k = b->stream_of[j];
        hipStream_t st = b->streams[k];
        if (!waited[k]) HIP_OK(hipStreamWaitEvent(st, b->head_done[w], 0));
        waited[k] = 1;
        if (b->timed) HIP_OK(launch_stamp(b->stamps + 1 + 2 * j, st));
        run_tail(b->plans[j], b->outs[j], st);
        if (b->timed) HIP_OK(launch_stamp(b->stamps + 2 + 2 * j, st));
      }
    }
    for (size_t k = 0; k < b->streams.size(); ++k) {
      HIP_OK(hipEventRecord(b->join[k], b->streams[k]));
      HIP_OK(hipStreamWaitEvent(origin, b->join[k], 0));
    }
    return;
  }
  if (b->grouped) {
    // wave w on worker stream w: its launches up to the final steps start
    // once wave w - 1's are done, then its shared final-step launches; every
    // launch is followed by its stamp
    HIP_OK(hipEventRecord(b->fork, origin));
    int slot = 1 + 2 * (int)b->plans.size();
    for (size_t w = 0; w < b->waves.size(); ++w) {
      hipStream_t st = b->streams[w];
      HIP_OK(hipStreamWaitEvent(st, w == 0 ? b->fork : b->head_done[w - 1], 0));
      for (auto &f : b->waves[w].steps) {
        f(st);
        if (b->timed) HIP_OK(launch_stamp(b->stamps + slot, st));
        ++slot;
      }
      HIP_OK(hipEventRecord(b->head_done[w], st));
      for (auto &f : b->waves[w].roots) {
        f(st);
        if (b->timed) HIP_OK(launch_stamp(b->stamps + slot, st));
        ++slot;
      }
      HIP_OK(hipEventRecord(b->join[w], st));
    }
    for (size_t w = 0; w < b->waves.size(); ++w) HIP_OK(hipStreamWaitEvent(origin, b->join[w], 0));
    return;
  }
  HIP_OK(hipEventRecord(b->fork, origin));
  for (auto st : b->streams) HIP_OK(hipStreamWaitEvent(st, b->fork, 0));
  for (int j : b->order) {
    hipStream_t st = b->streams[b->stream_of[j]];
    if (b->timed) HIP_OK(launch_stamp(b->stamps + 1 + 2 * j, st));
    execute(b->plans[j], b->outs[j], b->out_bytes[j], st);
    if (b->timed) HIP_OK(launch_stamp(b->stamps + 2 + 2 * j, st));
  }
  for (size_t k = 0; k < b->streams.size(); ++k) {
    HIP_OK(hipEventRecord(b->join[k], b->streams[k]));
    HIP_OK(hipStreamWaitEvent(origin, b->join[k], 0));
  }
}

static void multi_execute(Multi *b, hipStream_t s) {
  check_device(b->device);
  b->last_stream = s;
  b->ran = true;
  if (!b->use_graph) {
    multi_enqueue(b, s);
    return;
  }
  if (!b->exec) {
    HIP_OK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    bool ok = true;
    std::string msg;
    try {
      multi_enqueue(b, b->cap);
    } catch (const Error &e) {
      ok = false;
      msg = e.msg;
    }
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(b->cap, &g);
    if (!ok) {
      if (g) (void)hipGraphDestroy(g);
      fail(TQC_ERR_DEVICE, "capture of the jobs failed: %s", msg.c_str());
    }
    HIP_OK(ce);
    b->graph = g;
    HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  HIP_OK(hipGraphLaunch(b->exec, s));
}

// per-job start / end in milliseconds after the launch began (last call)
static void multi_times(Multi *b, double *start_ms, double *end_ms) {
  if (!b->timed) fail(TQC_ERR_INVALID_ARG, "the jobs were set up without timestamps");
  if (!b->ran) fail(TQC_ERR_INVALID_ARG, "the jobs have not run yet");
  check_device(b->device);
  HIP_OK(hipStreamSynchronize(b->last_stream));
  const size_t n = b->plans.size();
  std::vector<unsigned long long> st(std::max<size_t>(1 + 2 * n, (size_t)b->nslots));
  HIP_OK(hipMemcpy(st.data(), b->stamps, st.size() * 8, hipMemcpyDeviceToHost));
  for (size_t j = 0; j < n; ++j) {
    // grouped: every job starts with the launch and ends with the shared
    // launch that runs its final step; grouped heads: its own launches'
    // stamps, as without grouping
    const bool shared = b->grouped && !b->heads_only;
    const uint64_t s0 = shared ? 0 : 1 + 2 * j;
    const uint64_t e = shared ? (uint64_t)b->done_at[j] : 2 + 2 * j;
    if (start_ms) start_ms[j] = double((long long)(st[s0] - st[0])) * b->tick_ms;
    if (end_ms) end_ms[j] = double((long long)(st[e] - st[0])) * b->tick_ms;
  }
}

// ------------------------------------------------------------- cost model
struct CostModel {
  int device = -1;
  float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr, *d_partial = nullptr;
  float fmean[kFeat], fstd[kFeat];
  float tmean = 0.f, tstd = 1.f;
  int adam_step = 0;
  ~CostModel() {
    for (float *x : {d_theta, d_m, d_v, d_g, d_partial})
      if (x) (void)hipFree(x);
  }
};

// Raw features of one launch of a pairwise step (log2 sizes, roofline
// quantities, one-hot precision and tile).
static void shape_features(const StepShape &sh, Prec prec, tqc_dtype out_dtype, uint64_t slices,
                           float *f) {
  const double eb = prec_bytes(prec);
  double outb = eb;
  if (sh.root) outb = slices > 1 ? 16.0 : (out_dtype == TQC_F64 ? 8.0 : 4.0);
  const double bytes = eb * (std::ldexp(1.0, sh.lm) + std::ldexp(1.0, sh.ln)) * std::ldexp(1.0, sh.kpad) +
                       outb * std::ldexp(1.0, sh.lm + sh.ln);
  for (int i = 0; i < kFeat; ++i) f[i] = 0.f;
  f[0] = (float)sh.lm;
  f[1] = (float)sh.ln;
  f[2] = (float)sh.lk;
  f[3] = (float)sh.kpad;
  f[4] = (float)(sh.lm + sh.ln);
  f[5] = (float)(sh.lm + sh.ln + sh.lk);
  f[6] = (float)std::log2(bytes);
  f[7] = (float)sh.root;
  f[8] = (float)std::log2(outb);
  f[9 + (prec == Prec::F16X3 ? int(Prec::BF16X3) : int(prec))] = 1.f;  // same MFMA cost class
  f[13 + std::min(2, std::max(0, sh.tile))] = 1.f;
}

static CostModel *create_costmodel(uint64_t seed) {
  std::unique_ptr<CostModel> m(new CostModel());
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  m->device = dev;
  for (int i = 0; i < kFeat; ++i) {
    m->fmean[i] = 0.f;
    m->fstd[i] = 1.f;
  }
  std::vector<float> th(kParams, 0.f);
  std::mt19937_64 rng(seed ? seed : 12345);
  std::normal_distribution<float> nd(0.f, 1.f);
  // He initialisation of the two ReLU layers, small output layer
  for (int i = 0; i < kFeat * kHid; ++i) th[i] = nd(rng) * std::sqrt(2.f / kFeat);
  const int oW2 = kFeat * kHid + kHid;
  for (int i = 0; i < kHid * kHid; ++i) th[oW2 + i] = nd(rng) * std::sqrt(2.f / kHid);
  const int oW3 = oW2 + kHid * kHid + kHid;
  for (int i = 0; i < kHid; ++i) th[oW3 + i] = nd(rng) * std::sqrt(1.f / kHid);
  HIP_OK(hipMalloc((void **)&m->d_theta, kParams * 4));
  HIP_OK(hipMalloc((void **)&m->d_m, kParams * 4));
  HIP_OK(hipMalloc((void **)&m->d_v, kParams * 4));
  HIP_OK(hipMalloc((void **)&m->d_g, kParams * 4));
  HIP_OK(hipMalloc((void **)&m->d_partial, (size_t)kGradBlocks * 4 * kParams * 4));
  HIP_OK(hipMemcpy(m->d_theta, th.data(), kParams * 4, hipMemcpyHostToDevice));
  HIP_OK(hipMemset(m->d_m, 0, kParams * 4));
  HIP_OK(hipMemset(m->d_v, 0, kParams * 4));
  return m.release();
}

struct DevBuf {
  void *p = nullptr;
  explicit DevBuf(size_t bytes) { HIP_OK(hipMalloc(&p, bytes ? bytes : 4)); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

static void costmodel_forward_raw(CostModel *m, const float *X, int64_t n, float *y, hipStream_t s) {
  check_device(m->device);
  DevBuf dx(n * kFeat * 4), dy(n * 4);
  HIP_OK(hipMemcpyAsync(dx.p, X, n * kFeat * 4, hipMemcpyHostToDevice, s));
  HIP_OK(launch_mlp_forward(m->d_theta, (const float *)dx.p, n, (float *)dy.p, s));
  HIP_OK(hipMemcpyAsync(y, dy.p, n * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
}

static void costmodel_grad_raw(CostModel *m, const float *X, const float *t, int64_t n, float *g,
                               hipStream_t s) {
  check_device(m->device);
  DevBuf dx(n * kFeat * 4), dt(n * 4);
  HIP_OK(hipMemcpyAsync(dx.p, X, n * kFeat * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dt.p, t, n * 4, hipMemcpyHostToDevice, s));
  HIP_OK(launch_mlp_grad(m->d_theta, (const float *)dx.p, (const float *)dt.p, nullptr, n, m->d_partial,
                         m->d_g, s));
  HIP_OK(hipMemcpyAsync(g, m->d_g, kParams * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
}

static void costmodel_train(CostModel *m, const float *feats, const float *seconds, int64_t n,
                            const tqc_train_options &o, float *loss_out, hipStream_t s) {
  check_device(m->device);
  if (n < 2) fail(TQC_ERR_INVALID_ARG, "need at least two samples");
  // normalisation from the data
  for (int f = 0; f < kFeat; ++f) {
    double mu = 0, var = 0;
    for (int64_t i = 0; i < n; ++i) mu += feats[i * kFeat + f];
    mu /= n;
    for (int64_t i = 0; i < n; ++i) var += (feats[i * kFeat + f] - mu) * (feats[i * kFeat + f] - mu);
    var /= n;
    m->fmean[f] = (float)mu;
    m->fstd[f] = var > 1e-12 ? (float)std::sqrt(var) : 1.f;
  }
  std::vector<float> X(n * kFeat), T(n);
  double tm = 0, tv = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(seconds[i] > 0)) fail(TQC_ERR_INVALID_ARG, "sample %lld has a non-positive time", (long long)i);
    T[i] = (float)std::log((double)seconds[i]);
    tm += T[i];
  }
  tm /= n;
  for (int64_t i = 0; i < n; ++i) tv += (T[i] - tm) * (T[i] - tm);
  tv /= n;
  m->tmean = (float)tm;
  m->tstd = tv > 1e-12 ? (float)std::sqrt(tv) : 1.f;
  for (int64_t i = 0; i < n; ++i) {
    T[i] = (T[i] - m->tmean) / m->tstd;
    for (int f = 0; f < kFeat; ++f)
      X[i * kFeat + f] = (feats[i * kFeat + f] - m->fmean[f]) / m->fstd[f];
  }
  DevBuf dx(n * kFeat * 4), dt(n * 4), dperm(n * 4), dy(n * 4);
  HIP_OK(hipMemcpyAsync(dx.p, X.data(), n * kFeat * 4, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(dt.p, T.data(), n * 4, hipMemcpyHostToDevice, s));
  const int epochs = o.epochs > 0 ? o.epochs : 200;
  const int64_t bs = o.batch > 0 ? std::min<int64_t>(o.batch, n) : std::min<int64_t>(256, n);
  const float lr = o.lr > 0 ? o.lr : 3e-3f;
  std::mt19937_64 rng(o.seed ? o.seed : 7);
  std::vector<int32_t> perm(n);
  std::vector<float> y(n);
  for (int ep = 0; ep < epochs; ++ep) {
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    HIP_OK(hipMemcpyAsync(dperm.p, perm.data(), n * 4, hipMemcpyHostToDevice, s));
    for (int64_t b0 = 0; b0 + bs <= n; b0 += bs) {
      HIP_OK(launch_mlp_grad(m->d_theta, (const float *)dx.p, (const float *)dt.p,
                             (const int32_t *)dperm.p + b0, bs, m->d_partial, m->d_g, s));
      HIP_OK(launch_adam(m->d_theta, m->d_g, m->d_m, m->d_v, lr, 0.9f, 0.999f, 1e-8f, ++m->adam_step, s));
    }
    if (loss_out) {
      HIP_OK(launch_mlp_forward(m->d_theta, (const float *)dx.p, n, (float *)dy.p, s));
      HIP_OK(hipMemcpyAsync(y.data(), dy.p, n * 4, hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      double L = 0;
      for (int64_t i = 0; i < n; ++i) L += double(y[i] - T[i]) * double(y[i] - T[i]);
      loss_out[ep] = (float)(L / n);
    }
  }
  HIP_OK(hipStreamSynchronize(s));
}

// predicted seconds of launches described by raw feature rows
static void costmodel_predict(CostModel *m, const float *feats, int64_t n, double *sec, hipStream_t s) {
  std::vector<float> X(n * kFeat), y(n);
  for (int64_t i = 0; i < n; ++i)
    for (int f = 0; f < kFeat; ++f) X[i * kFeat + f] = (feats[i * kFeat + f] - m->fmean[f]) / m->fstd[f];
  costmodel_forward_raw(m, X.data(), n, y.data(), s);
  for (int64_t i = 0; i < n; ++i) sec[i] = std::exp((double)y[i] * m->tstd + m->tmean);
}

// Rank candidate orders with the model; returns the best order.
static std::vector<int> mlp_choose_order(Network *net, Prec prec, tqc_dtype out, const std::vector<int> &sliced,
                                         const std::vector<int> &fixed_q, CostModel *m, int count,
                                         uint64_t seed, double *best_score, hipStream_t s,
                                         const std::vector<int> *roofline_order = nullptr) {
  auto orders = sample_orders(net, prec, out, sliced, fixed_q, std::max(2, count), seed);
  // the roofline planner's own order competes too: the model only replaces
  // it where it predicts a faster one
  if (roofline_order && !roofline_order->empty()) orders.insert(orders.begin(), *roofline_order);
  const uint64_t slices = 1ull << (2 * sliced.size());
  std::vector<float> F;
  std::vector<double> mult;
  std::vector<size_t> row0(orders.size() + 1, 0);
  for (size_t c = 0; c < orders.size(); ++c) {
    auto sh = order_shapes(net, prec, sliced, fixed_q, orders[c]);
    for (auto &x : sh) {
      float f[kFeat];
      shape_features(x, prec, out, slices, f);
      F.insert(F.end(), f, f + kFeat);
      mult.push_back(x.slice_dep ? double(slices) : 1.0);
    }
    row0[c + 1] = mult.size();
  }
  std::vector<double> sec(mult.size());
  if (!mult.empty()) costmodel_predict(m, F.data(), (int64_t)mult.size(), sec.data(), s);
  size_t best = 0;
  double bs = 1e300;
  for (size_t c = 0; c < orders.size(); ++c) {
    double sc = 0;
    for (size_t r = row0[c]; r < row0[c + 1]; ++r) sc += sec[r] * mult[r];
    if (sc < bs) {
      bs = sc;
      best = c;
    }
  }
  if (best_score) *best_score = bs;
  return orders[best];
}

// ---------------------------------------------- measured time as the judge
// The learned model (or, without one, the roofline model) only shortlists:
// the roofline planner's plan and the `count` best-ranked other orders are
// each run on the device at full size, their median time over `reps` runs
// is measured with HIP events, and every form other than float64 is checked
// against a float64 run of the roofline plan (max |P - P_ref| / max |P_ref|
// over every output entry).  The fastest plan within the error bound wins;
// the roofline plan is the fallback when no other candidate passes.
struct Measured {
  double seconds = 0, rel_err = -1;
};

static void finish_tiles(Plan *p, int tile_policy) {
  for (Step &st : p->steps) st.tile = pick_tile(p, st);
  if (tile_policy == 1) apply_tuned_tiles(p);
}

static std::vector<int> order_of(const Plan *p) {
  std::vector<int> o;
  for (const Step &st : p->steps) {
    o.push_back(st.a);
    o.push_back(st.b);
  }
  return o;
}

static Measured measure_plan(Plan *p, void *out, const double *ref, unsigned long long *errbits, int reps,
                             hipStream_t s) {
  const uint64_t entries = 1ull << p->out_bits;
  const uint64_t bytes = entries * (p->out_dtype == TQC_F64 ? 8 : 4);
  execute(p, out, bytes, s);  // warm-up: workspace, transform, caches
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto &e : ev) HIP_OK(hipEventCreate(&e));
  for (int r = 0; r < reps; ++r) {
    HIP_OK(hipEventRecord(ev[2 * r], s));
    execute(p, out, bytes, s);
    HIP_OK(hipEventRecord(ev[2 * r + 1], s));
  }
  HIP_OK(hipStreamSynchronize(s));
  std::vector<double> ms(reps);
  for (int r = 0; r < reps; ++r) {
    float t = 0;
    HIP_OK(hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]));
    ms[r] = t;
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  std::sort(ms.begin(), ms.end());
  Measured m;
  m.seconds = ms[reps / 2] * 1e-3;
  if (ref) {
    HIP_OK(launch_zero_u64(errbits, 2, s));
    HIP_OK(launch_max_abs_diff(out, p->out_dtype == TQC_F32 ? 1 : 0, ref, entries, errbits, s));
    unsigned long long h[2];
    HIP_OK(hipMemcpyAsync(h, errbits, 16, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double d, r;
    std::memcpy(&d, &h[0], 8);
    std::memcpy(&r, &h[1], 8);
    m.rel_err = r > 0 ? d / r : d;
  }
  return m;
}

static Plan *plan_measured(Network *net, const tqc_plan_options &opt) {
  auto t0 = std::chrono::steady_clock::now();
  CostModel *model = reinterpret_cast<CostModel *>(opt.cost_model);
  const int count = opt.num_measured > 0 ? opt.num_measured : 4;
  const int reps = 5;
  const double tol = opt.max_rel_error > 0 ? opt.max_rel_error : 1e-6;
  tqc_plan_options o1 = opt;
  o1.cost_kind = TQC_COST_FLOPBYTE;
  o1.cost_model = nullptr;
  std::unique_ptr<Plan> best(build_plan(net, o1));
  finish_tiles(best.get(), opt.tile_policy);
  const std::vector<int> p0_order = order_of(best.get());
  // shortlist: the best-ranked sampled orders other than the roofline one
  std::vector<std::vector<int>> shortlist;
  if (net->m >= 3) {
    auto orders = sample_orders(net, best->prec, best->out_dtype, best->sliced, best->fixed_q,
                                opt.num_candidates > 0 ? opt.num_candidates : 1000, opt.seed);
    std::vector<double> score(orders.size(), 0.0);
    if (model) {
      const uint64_t slices = 1ull << (2 * best->sliced.size());
      std::vector<float> F;
      std::vector<double> mult;
      std::vector<size_t> row0(orders.size() + 1, 0);
      for (size_t c = 0; c < orders.size(); ++c) {
        for (auto &x : order_shapes(net, best->prec, best->sliced, best->fixed_q, orders[c])) {
          float f[kFeat];
          shape_features(x, best->prec, best->out_dtype, slices, f);
          F.insert(F.end(), f, f + kFeat);
          mult.push_back(x.slice_dep ? double(slices) : 1.0);
        }
        row0[c + 1] = mult.size();
      }
      std::vector<double> sec(mult.size());
      if (!mult.empty()) costmodel_predict(model, F.data(), (int64_t)mult.size(), sec.data(), nullptr);
      for (size_t c = 0; c < orders.size(); ++c)
        for (size_t r = row0[c]; r < row0[c + 1]; ++r) score[c] += sec[r] * mult[r];
    } else {
      for (size_t c = 0; c < orders.size(); ++c) {
        tqc_plan_options oc = o1;
        oc.num_order_steps = (int32_t)orders[c].size() / 2;
        oc.order = orders[c].data();
        oc.num_sliced = (int32_t)best->sliced.size();
        oc.sliced_cuts = best->sliced.data();
        oc.mem_budget_bytes = 0;
        std::unique_ptr<Plan> pc(build_plan(net, oc));
        score[c] = pc->stats.predicted_seconds;
      }
    }
    std::vector<size_t> idx(orders.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return score[a] < score[b]; });
    for (size_t i : idx) {
      if ((int)shortlist.size() >= count) break;
      if (orders[i] == p0_order) continue;
      if (std::find(shortlist.begin(), shortlist.end(), orders[i]) != shortlist.end()) continue;
      shortlist.push_back(orders[i]);
    }
  }
  // device measurement on a private stream
  upload(net);
  check_device(net->device);
  hipStream_t s = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct Cleanup {
    std::vector<void *> bufs;
    hipStream_t s;
    ~Cleanup() {
      if (s) (void)hipStreamSynchronize(s);
      for (void *b : bufs) (void)hipFree(b);
      if (s) (void)hipStreamDestroy(s);
    }
  } cl{{}, s};
  const uint64_t entries = 1ull << best->out_bits;
  void *out = nullptr;
  HIP_OK(hipMalloc(&out, entries * (best->out_dtype == TQC_F64 ? 8 : 4)));
  cl.bufs.push_back(out);
  unsigned long long *errbits = nullptr;
  HIP_OK(hipMalloc((void **)&errbits, 16));
  cl.bufs.push_back(errbits);
  double *ref = nullptr;
  if (best->prec != Prec::F64) {
    tqc_plan_options orf = o1;
    orf.precision = TQC_FP64;
    orf.out_dtype = TQC_F64;
    orf.num_order_steps = (int32_t)p0_order.size() / 2;
    orf.order = p0_order.data();
    orf.num_sliced = (int32_t)best->sliced.size();
    orf.sliced_cuts = best->sliced.data();
    orf.mem_budget_bytes = 0;
    std::unique_ptr<Plan> pr(build_plan(net, orf));
    finish_tiles(pr.get(), 0);
    HIP_OK(hipMalloc((void **)&ref, entries * 8));
    cl.bufs.push_back(ref);
    execute(pr.get(), ref, entries * 8, s);
    HIP_OK(hipStreamSynchronize(s));
  }
  const Measured m0 = measure_plan(best.get(), out, ref, errbits, reps, s);
  Measured bm = m0;
  int measured = 1;
  for (const auto &ord : shortlist) {
    tqc_plan_options oc = o1;
    oc.num_order_steps = (int32_t)ord.size() / 2;
    oc.order = ord.data();
    oc.num_sliced = (int32_t)best->sliced.size();
    oc.sliced_cuts = best->sliced.data();
    oc.mem_budget_bytes = 0;
    std::unique_ptr<Plan> pc(build_plan(net, oc));
    finish_tiles(pc.get(), opt.tile_policy);
    if (opt.mem_budget_bytes && pc->stats.workspace_bytes > opt.mem_budget_bytes) continue;
    const Measured mc = measure_plan(pc.get(), out, ref, errbits, reps, s);
    ++measured;
    const bool ok = mc.rel_err < 0 || mc.rel_err <= tol;
    const bool best_ok = bm.rel_err < 0 || bm.rel_err <= tol;
    if (ok && (!best_ok || mc.seconds < bm.seconds)) {
      best = std::move(pc);
      bm = mc;
    }
  }
  best->stats.measured_seconds = bm.seconds;
  best->stats.checked_rel_error = bm.rel_err;
  best->stats.fallback_measured_seconds = m0.seconds;
  best->stats.num_measured = measured;
  best->stats.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return best.release();
}

}  // namespace tqc

using namespace tqc;

struct tqc_network_s : Network {};
struct tqc_plan_s : Plan {};

// ---------------------------------------------------------- plan blobs
// A plan's decisions (Sec. III-E: the contraction order and the sliced cuts;
// the fixed-qubit slice, the form and every step's tile) as a byte string,
// together with the structure of the network it was made for (qubits, cut
// ends, each tensor's basis, cut list and output qubits).  Tensor values are
// not part of it: a plan depends only on the structure, so a stored plan
// serves every network of that structure.  Little-endian; the last 8 bytes
// are an FNV-1a hash of the rest.
namespace {
constexpr char kPlanMagic[8] = {'T', 'Q', 'C', 'P', 'L', 'A', 'N', '1'};

struct BlobWriter {
  std::vector<unsigned char> b;
  void put(const void *p, size_t n) { b.insert(b.end(), (const unsigned char *)p, (const unsigned char *)p + n); }
  void i32(int32_t v) { put(&v, 4); }
  void u64(uint64_t v) { put(&v, 8); }
  void f64(double v) { put(&v, 8); }
};

struct BlobReader {
  const unsigned char *p;
  size_t n, at = 0;
  void get(void *dst, size_t k) {
    if (k > n - at) fail(TQC_ERR_INVALID_ARG, "plan blob truncated at byte %zu", at);
    std::memcpy(dst, p + at, k);
    at += k;
  }
  int32_t i32() { int32_t v; get(&v, 4); return v; }
  uint64_t u64() { uint64_t v; get(&v, 8); return v; }
  double f64() { double v; get(&v, 8); return v; }
};

uint64_t fnv1a(const unsigned char *p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

void write_structure(BlobWriter &w, const Network &net) {
  w.i32(net.n);
  w.i32(net.m);
  w.i32(net.K);
  for (const tqc_cut &c : net.cuts) {
    w.i32(c.upstream);
    w.i32(c.downstream);
  }
  for (const TensorIn &t : net.t) {
    w.i32((int32_t)t.basis);
    w.i32((int32_t)t.cuts.size());
    for (int c : t.cuts) w.i32(c);
    w.i32((int32_t)t.outputs.size());
    for (int q : t.outputs) w.i32(q);
  }
}

std::vector<unsigned char> serialize_plan(const Plan &p) {
  BlobWriter w;
  w.put(kPlanMagic, 8);
  write_structure(w, *p.net);
  w.i32((int32_t)p.prec);
  w.i32((int32_t)p.out_dtype);
  w.i32(p.tile_policy);
  w.i32((int32_t)p.fixed_q.size());
  for (size_t i = 0; i < p.fixed_q.size(); ++i) {
    w.i32(p.fixed_q[i]);
    w.i32(p.fixed_v[i]);
  }
  w.i32((int32_t)p.sliced.size());
  for (int c : p.sliced) w.i32(c);
  w.i32((int32_t)p.steps.size());
  for (const Step &st : p.steps) {
    w.i32(st.a);
    w.i32(st.b);
    w.i32(st.tile);
  }
  w.f64(p.stats.predicted_seconds);
  w.u64(fnv1a(w.b.data(), w.b.size()));
  return w.b;
}

Plan *deserialize_plan(Network *net, const unsigned char *buf, size_t len) {
  if (len < 16) fail(TQC_ERR_INVALID_ARG, "plan blob of %zu bytes", len);
  uint64_t h;
  std::memcpy(&h, buf + len - 8, 8);
  if (h != fnv1a(buf, len - 8)) fail(TQC_ERR_INVALID_ARG, "plan blob checksum mismatch");
  if (std::memcmp(buf, kPlanMagic, 8) != 0) fail(TQC_ERR_INVALID_ARG, "not a plan blob");
  // the structure must match byte for byte
  BlobWriter mine;
  write_structure(mine, *net);
  if (len - 16 < mine.b.size() || std::memcmp(buf + 8, mine.b.data(), mine.b.size()) != 0)
    fail(TQC_ERR_TOPOLOGY, "the plan was made for a network of another structure");
  BlobReader r{buf, len - 8, 8 + mine.b.size()};
  tqc_plan_options o;
  tqc_plan_options_default(&o);
  o.precision = (tqc_precision)r.i32();
  o.out_dtype = (tqc_dtype)r.i32();
  o.tile_policy = r.i32();
  const int nf = r.i32();
  if (nf < 0 || nf > net->n) fail(TQC_ERR_INVALID_ARG, "plan blob: %d fixed qubits", nf);
  std::vector<int32_t> fq(nf), fv(nf);
  for (int i = 0; i < nf; ++i) {
    fq[i] = r.i32();
    fv[i] = r.i32();
  }
  const int ns = r.i32();
  if (ns < 0 || ns > net->K) fail(TQC_ERR_INVALID_ARG, "plan blob: %d sliced cuts", ns);
  std::vector<int32_t> sl(ns);
  for (int i = 0; i < ns; ++i) sl[i] = r.i32();
  const int nsteps = r.i32();
  if (nsteps != std::max(0, net->m - 1)) fail(TQC_ERR_INVALID_ARG, "plan blob: %d steps for %d tensors", nsteps, net->m);
  std::vector<int32_t> order(2 * nsteps), tiles(nsteps);
  for (int i = 0; i < nsteps; ++i) {
    order[2 * i] = r.i32();
    order[2 * i + 1] = r.i32();
    tiles[i] = r.i32();
    if (tiles[i] < 0 || tiles[i] > 2) fail(TQC_ERR_INVALID_ARG, "plan blob: tile %d", tiles[i]);
  }
  const double predicted = r.f64();
  if (r.at != r.n) fail(TQC_ERR_INVALID_ARG, "plan blob has %zu trailing bytes", r.n - r.at);
  o.num_fixed = nf;
  o.fixed_qubits = fq.data();
  o.fixed_values = fv.data();
  o.num_sliced = ns;
  o.sliced_cuts = sl.data();
  o.num_order_steps = nsteps;
  o.order = order.data();
  std::unique_ptr<Plan> p(build_plan(net, o));
  for (int i = 0; i < nsteps; ++i) p->steps[i].tile = tiles[i];
  p->stats.predicted_seconds = predicted;
  return p.release();
}
}  // namespace

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
    Plan *p = nullptr;
    if (opt->cost_kind == TQC_COST_MEASURED && opt->num_order_steps <= 0) {
      p = plan_measured(reinterpret_cast<Network *>(net), *opt);
      *out = reinterpret_cast<tqc_plan_t>(p);
      return;
    }
    if (opt->cost_kind == TQC_COST_MLP && opt->num_order_steps <= 0) {
      if (!opt->cost_model) fail(TQC_ERR_INVALID_ARG, "TQC_COST_MLP needs a cost model");
      auto t0 = std::chrono::steady_clock::now();
      // slicing from the roofline planner, order from the learned model
      tqc_plan_options o1 = *opt;
      o1.cost_kind = TQC_COST_FLOPBYTE;
      std::unique_ptr<Plan> p0(build_plan(reinterpret_cast<Network *>(net), o1));
      double score = 0;
      std::vector<int> p0_order;
      for (const Step &st : p0->steps) {
        p0_order.push_back(st.a);
        p0_order.push_back(st.b);
      }
      std::vector<int> order = mlp_choose_order(
          reinterpret_cast<Network *>(net), p0->prec, p0->out_dtype, p0->sliced, p0->fixed_q,
          reinterpret_cast<CostModel *>(opt->cost_model),
          opt->num_candidates > 0 ? opt->num_candidates : 1000, opt->seed, &score, nullptr, &p0_order);
      tqc_plan_options o2 = o1;
      o2.num_order_steps = (int32_t)order.size() / 2;
      o2.order = order.data();
      o2.num_sliced = (int32_t)p0->sliced.size();
      o2.sliced_cuts = p0->sliced.data();
      p = build_plan(reinterpret_cast<Network *>(net), o2);
      p->stats.predicted_seconds = score;
      p->stats.plan_seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } else {
      p = build_plan(reinterpret_cast<Network *>(net), *opt);
    }
    for (Step &st : p->steps) st.tile = pick_tile(p, st);
    if (opt->tile_policy == 1) apply_tuned_tiles(p);
    *out = reinterpret_cast<tqc_plan_t>(p);
  });
}

void tqc_plan_destroy(tqc_plan_t plan) { delete reinterpret_cast<Plan *>(plan); }

tqc_status tqc_plan_get_stats(tqc_plan_t plan, tqc_plan_stats *st) {
  return guarded([&] {
    if (!plan || !st) fail(TQC_ERR_INVALID_ARG, "null argument");
    const Plan *p = reinterpret_cast<Plan *>(plan);
    *st = p->stats;
    st->precision = (int32_t)p->prec;
    st->out_dtype = (int32_t)p->out_dtype;
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

tqc_status tqc_execute_summary(tqc_plan_t plan, void *out, uint64_t out_bytes, int32_t k,
                               uint64_t *top_idx, double *top_val, double *total, double *phase_ms,
                               int32_t num_phases, void *stream) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p) fail(TQC_ERR_INVALID_ARG, "null plan");
    if (phase_ms) {
      const int need = 3 + (int)p->steps.size();
      if (num_phases < need) fail(TQC_ERR_SHAPE, "phase_ms needs %d entries", need);
      Timing tm;
      tm.s = (hipStream_t)stream;
      execute_summary(p, out, out_bytes, k, top_idx, top_val, total, (hipStream_t)stream, &tm);
      tm.collect(phase_ms, num_phases);
    } else {
      execute_summary(p, out, out_bytes, k, top_idx, top_val, total, (hipStream_t)stream, nullptr);
    }
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

static void check_topk_args(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k, const uint64_t *idx_out,
                            const double *val_out) {
  if (!probs || !idx_out || !val_out) fail(TQC_ERR_INVALID_ARG, "null argument");
  if (dtype != TQC_F32 && dtype != TQC_F64) fail(TQC_ERR_INVALID_ARG, "dtype");
  if (k < 1 || k > 4096 || (uint64_t)k > len)
    fail(TQC_ERR_INVALID_ARG, "k = %d for length %llu", k, (unsigned long long)len);
}

static void check_marginal_args(const void *probs, tqc_dtype dtype, int32_t num_qubits, int32_t num_keep,
                                const int32_t *keep, const double *out) {
  if (!probs || !out || (num_keep > 0 && !keep)) fail(TQC_ERR_INVALID_ARG, "null argument");
  if (dtype != TQC_F32 && dtype != TQC_F64) fail(TQC_ERR_INVALID_ARG, "dtype");
  if (num_qubits < 0 || num_qubits > 40) fail(TQC_ERR_INVALID_ARG, "num_qubits %d", num_qubits);
  if (num_keep < 0 || num_keep > 24 || num_keep > num_qubits) fail(TQC_ERR_INVALID_ARG, "num_keep %d", num_keep);
  for (int i = 0; i < num_keep; ++i) {
    if (keep[i] < 0 || keep[i] >= num_qubits) fail(TQC_ERR_INVALID_ARG, "keep qubit %d", keep[i]);
    for (int j = 0; j < i; ++j)
      if (keep[j] == keep[i]) fail(TQC_ERR_INVALID_ARG, "keep qubit %d twice", keep[i]);
  }
}

tqc_status tqc_topk(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k, uint64_t *idx_out,
                    double *val_out, void *stream) {
  return guarded([&] {
    check_topk_args(probs, dtype, len, k, idx_out, val_out);
    const uint64_t sb = topk_scratch_bytes(len, k);
    ScratchLease lease = stream_scratch(sb, (hipStream_t)stream);
    HIP_OK(launch_topk(probs, dtype == TQC_F32 ? 1 : 0, len, k, idx_out, val_out, lease.ptr, sb,
                       (hipStream_t)stream));
  });
}

tqc_status tqc_topk_noalloc(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k, uint64_t *idx_out,
                            double *val_out, void *stream) {
  return guarded([&] {
    check_topk_args(probs, dtype, len, k, idx_out, val_out);
    const uint64_t sb = topk_scratch_bytes(len, k);
    if (sb > kNoAllocScratchBytes)
      fail(TQC_ERR_INVALID_ARG, "top-k of %llu entries needs %llu scratch bytes; the fixed scratch holds %llu",
           (unsigned long long)len, (unsigned long long)sb, (unsigned long long)kNoAllocScratchBytes);
    void *ptr = noalloc_scratch();
    HIP_OK(launch_topk(probs, dtype == TQC_F32 ? 1 : 0, len, k, idx_out, val_out, ptr, sb, (hipStream_t)stream));
  });
}

tqc_status tqc_topk_workspace_bytes(uint64_t len, int32_t k, uint64_t *bytes) {
  return guarded([&] {
    if (!bytes) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (k < 1 || k > 4096 || (uint64_t)k > len)
      fail(TQC_ERR_INVALID_ARG, "k = %d for length %llu", k, (unsigned long long)len);
    *bytes = topk_scratch_bytes(len, k);
  });
}

tqc_status tqc_topk_ws(const void *probs, tqc_dtype dtype, uint64_t len, int32_t k, uint64_t *idx_out,
                       double *val_out, void *workspace, uint64_t ws_bytes, void *stream) {
  return guarded([&] {
    check_topk_args(probs, dtype, len, k, idx_out, val_out);
    if (!workspace || ((uintptr_t)workspace & 255)) fail(TQC_ERR_INVALID_ARG, "workspace null or not 256-byte aligned");
    const uint64_t sb = topk_scratch_bytes(len, k);
    if (ws_bytes < sb)
      fail(TQC_ERR_SHAPE, "workspace holds %llu bytes, needs %llu", (unsigned long long)ws_bytes,
           (unsigned long long)sb);
    HIP_OK(launch_topk(probs, dtype == TQC_F32 ? 1 : 0, len, k, idx_out, val_out, workspace, sb,
                       (hipStream_t)stream));
  });
}

tqc_status tqc_marginal(const void *probs, tqc_dtype dtype, int32_t num_qubits, int32_t num_keep,
                        const int32_t *keep, double *out, void *stream) {
  return guarded([&] {
    check_marginal_args(probs, dtype, num_qubits, num_keep, keep, out);
    const uint64_t sb = marginal_scratch_bytes(num_qubits, num_keep);
    ScratchLease lease = stream_scratch(sb, (hipStream_t)stream);
    HIP_OK(launch_marginal(probs, dtype == TQC_F32 ? 1 : 0, num_qubits, num_keep, keep, out, lease.ptr, sb,
                           (hipStream_t)stream));
  });
}

tqc_status tqc_marginal_workspace_bytes(int32_t num_qubits, int32_t num_keep, uint64_t *bytes) {
  return guarded([&] {
    if (!bytes) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (num_qubits < 0 || num_qubits > 40 || num_keep < 0 || num_keep > 24 || num_keep > num_qubits)
      fail(TQC_ERR_INVALID_ARG, "num_qubits %d, num_keep %d", num_qubits, num_keep);
    *bytes = marginal_scratch_bytes(num_qubits, num_keep);
  });
}

tqc_status tqc_marginal_ws(const void *probs, tqc_dtype dtype, int32_t num_qubits, int32_t num_keep,
                           const int32_t *keep, double *out, void *workspace, uint64_t ws_bytes, void *stream) {
  return guarded([&] {
    check_marginal_args(probs, dtype, num_qubits, num_keep, keep, out);
    if (!workspace || ((uintptr_t)workspace & 255)) fail(TQC_ERR_INVALID_ARG, "workspace null or not 256-byte aligned");
    const uint64_t sb = marginal_scratch_bytes(num_qubits, num_keep);
    if (ws_bytes < sb)
      fail(TQC_ERR_SHAPE, "workspace holds %llu bytes, needs %llu", (unsigned long long)ws_bytes,
           (unsigned long long)sb);
    HIP_OK(launch_marginal(probs, dtype == TQC_F32 ? 1 : 0, num_qubits, num_keep, keep, out, workspace, sb,
                           (hipStream_t)stream));
  });
}

tqc_status tqc_plan_workspace_bytes(tqc_plan_t plan, uint64_t *bytes) {
  return guarded([&] {
    if (!plan || !bytes) fail(TQC_ERR_INVALID_ARG, "null argument");
    *bytes = plan_layout(reinterpret_cast<Plan *>(plan)).total;
  });
}

tqc_status tqc_plan_set_workspace(tqc_plan_t plan, void *workspace, uint64_t ws_bytes, void *stream) {
  return guarded([&] {
    if (!plan) fail(TQC_ERR_INVALID_ARG, "null plan");
    bind_workspace(reinterpret_cast<Plan *>(plan), workspace, ws_bytes, (hipStream_t)stream);
  });
}

tqc_status tqc_plan_serialize(tqc_plan_t plan, void *buf, uint64_t *len) {
  return guarded([&] {
    if (!plan || !len) fail(TQC_ERR_INVALID_ARG, "null argument");
    const std::vector<unsigned char> b = serialize_plan(*reinterpret_cast<Plan *>(plan));
    if (buf) {
      if (*len < b.size())
        fail(TQC_ERR_SHAPE, "buffer holds %llu bytes, the plan needs %zu", (unsigned long long)*len, b.size());
      std::memcpy(buf, b.data(), b.size());
    }
    *len = b.size();
  });
}

tqc_status tqc_plan_deserialize(tqc_network_t net, const void *buf, uint64_t len, tqc_plan_t *out) {
  return guarded([&] {
    if (!net || !buf || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    Plan *p = deserialize_plan(reinterpret_cast<Network *>(net), (const unsigned char *)buf, (size_t)len);
    *out = reinterpret_cast<tqc_plan_t>(p);
  });
}

struct tqc_batch_s : Batch {};
struct tqc_multi_s : Multi {};

tqc_status tqc_find_cuts(int32_t num_qubits, int32_t num_gates, const int32_t *gate_qubits, int32_t w_max,
                         int32_t s_max, int32_t k_t, double q_max, int32_t *labels, int32_t *num_parts) {
  return guarded([&] {
    if (num_qubits < 1 || num_gates < 0 || (num_gates && (!gate_qubits || !labels)) || !num_parts)
      fail(TQC_ERR_INVALID_ARG, "bad circuit arguments");
    if (w_max < 1 || s_max < 1 || k_t < 1 || !(q_max >= 0)) fail(TQC_ERR_INVALID_ARG, "thresholds must be positive");
    *num_parts = find_cuts(num_qubits, num_gates, gate_qubits, w_max, s_max, k_t, q_max, labels);
  });
}

tqc_status tqc_hss_select(tqc_network_t netp, uint64_t s_max, int32_t *counts, int32_t *states,
                          uint64_t states_cap, double *norms, uint64_t norms_cap, void *stream) {
  return guarded([&] {
    Network *net = reinterpret_cast<Network *>(netp);
    if (!net || !counts || !states) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (s_max < 1) fail(TQC_ERR_INVALID_ARG, "s_max must be at least 1");
    std::vector<std::vector<double>> nv;
    hss_norms(net, nv, (hipStream_t)stream);
    const auto sel = hss_choose(nv, s_max);
    uint64_t total = 0, ncols = 0;
    for (int j = 0; j < net->m; ++j) {
      total += sel[j].size();
      ncols += nv[j].size();
    }
    if (total > states_cap) fail(TQC_ERR_SHAPE, "states holds %llu entries, needs %llu",
                                 (unsigned long long)states_cap, (unsigned long long)total);
    if (norms && norms_cap < ncols) fail(TQC_ERR_SHAPE, "norms holds %llu entries, needs %llu",
                                         (unsigned long long)norms_cap, (unsigned long long)ncols);
    uint64_t at = 0, an = 0;
    for (int j = 0; j < net->m; ++j) {
      counts[j] = (int32_t)sel[j].size();
      for (int32_t v : sel[j]) states[at++] = v;
      if (norms)
        for (double v : nv[j]) norms[an++] = v;
    }
  });
}

tqc_status tqc_network_select_states(tqc_network_t netp, const int32_t *counts, const int32_t *states, void *stream,
                                     tqc_network_t *out) {
  return guarded([&] {
    Network *net = reinterpret_cast<Network *>(netp);
    if (!net || !counts || !states || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    *out = reinterpret_cast<tqc_network_t>(select_states_network(net, counts, states, (hipStream_t)stream));
  });
}

tqc_status tqc_multi_create(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                            const uint64_t *out_bytes, int32_t use_graph, int32_t num_streams, int32_t timed,
                            void *stream, tqc_multi_t *out) {
  return guarded([&] {
    if (!out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    Multi *m = create_multi(num_jobs, reinterpret_cast<Plan *const *>(plans), outs, out_bytes, use_graph,
                            num_streams, timed, (hipStream_t)stream);
    *out = reinterpret_cast<tqc_multi_t>(static_cast<tqc_multi_s *>(m));
  });
}

tqc_status tqc_multi_create_ex(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                               const uint64_t *out_bytes, const tqc_multi_options *opt, void *stream,
                               tqc_multi_t *out) {
  return guarded([&] {
    if (!out || !opt) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    Multi *m = create_multi(num_jobs, reinterpret_cast<Plan *const *>(plans), outs, out_bytes, opt->use_graph,
                            opt->num_streams, opt->timed, (hipStream_t)stream, opt->grouped,
                            opt->waves > 0 ? opt->waves : 1);
    *out = reinterpret_cast<tqc_multi_t>(static_cast<tqc_multi_s *>(m));
  });
}

tqc_status tqc_multi_info(tqc_multi_t multi, int32_t *launches, int32_t *shared_root_jobs,
                          int32_t *shared_root_launches) {
  return guarded([&] {
    if (!multi) fail(TQC_ERR_INVALID_ARG, "null argument");
    const Multi *m = static_cast<Multi *>(multi);
    int32_t nl = 0;
    for (auto &w : m->waves) nl += (int32_t)(w.steps.size() + w.roots.size());
    if (launches) *launches = m->grouped ? nl : -1;  // grouped heads: the shared launches only
    if (shared_root_jobs) *shared_root_jobs = m->shared_root_jobs;
    if (shared_root_launches) *shared_root_launches = m->shared_roots;
  });
}

tqc_status tqc_multi_execute(tqc_multi_t multi, void *stream) {
  return guarded([&] {
    if (!multi) fail(TQC_ERR_INVALID_ARG, "null argument");
    multi_execute(static_cast<Multi *>(multi), (hipStream_t)stream);
  });
}

tqc_status tqc_multi_job_times(tqc_multi_t multi, double *start_ms, double *end_ms) {
  return guarded([&] {
    if (!multi) fail(TQC_ERR_INVALID_ARG, "null argument");
    multi_times(static_cast<Multi *>(multi), start_ms, end_ms);
  });
}

void tqc_multi_destroy(tqc_multi_t multi) {
  if (multi) delete static_cast<Multi *>(static_cast<tqc_multi_s *>(multi));
}

tqc_status tqc_batch_create(int32_t num_jobs, const tqc_plan_t *plans, void *const *outs,
                            const uint64_t *out_bytes, const tqc_batch_options *opt, void *stream,
                            tqc_batch_t *out) {
  return guarded([&] {
    if (!plans || !outs || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    tqc_batch_options o{};
    o.use_graph = 1;
    if (opt) o = *opt;
    Batch *b = create_batch(num_jobs, reinterpret_cast<Plan *const *>(plans), outs, out_bytes, o,
                            (hipStream_t)stream);
    *out = reinterpret_cast<tqc_batch_t>(b);
  });
}

tqc_status tqc_batch_validate(int32_t num_jobs, const tqc_plan_t *plans, const uint64_t *out_bytes,
                              char *report, uint64_t report_cap) {
  return guarded([&] {
    if (num_jobs < 1 || !plans) fail(TQC_ERR_INVALID_ARG, "no jobs");
    for (int j = 0; j < num_jobs; ++j)
      if (!plans[j]) fail(TQC_ERR_INVALID_ARG, "job %d: null plan", j);
    const std::string r = batch_emulate(num_jobs, reinterpret_cast<Plan *const *>(plans), out_bytes, 1ull << 32);
    if (report && report_cap) {
      const size_t n = std::min<size_t>(r.size(), report_cap - 1);
      std::memcpy(report, r.data(), n);
      report[n] = 0;
    }
    if (!r.empty()) fail(TQC_ERR_INTERNAL, "batch emulation: %s", r.c_str());
  });
}

tqc_status tqc_batch_execute(tqc_batch_t batch, void *stream) {
  return guarded([&] {
    if (!batch) fail(TQC_ERR_INVALID_ARG, "null batch");
    batch_execute(reinterpret_cast<Batch *>(batch), (hipStream_t)stream);
  });
}

tqc_status tqc_batch_execute_sequential(tqc_batch_t batch, void *stream, double *job_ms) {
  return guarded([&] {
    if (!batch) fail(TQC_ERR_INVALID_ARG, "null batch");
    batch_sequential(reinterpret_cast<Batch *>(batch), (hipStream_t)stream, job_ms);
  });
}

tqc_status tqc_batch_job_times(tqc_batch_t batch, double *start_ms, double *end_ms, uint32_t *error) {
  return guarded([&] {
    if (!batch) fail(TQC_ERR_INVALID_ARG, "null batch");
    batch_times(reinterpret_cast<Batch *>(batch), start_ms, end_ms, error);
  });
}

tqc_status tqc_batch_info(tqc_batch_t batch, uint64_t *items, int32_t *units, int32_t *grid) {
  return guarded([&] {
    Batch *b = reinterpret_cast<Batch *>(batch);
    if (!b) fail(TQC_ERR_INVALID_ARG, "null batch");
    if (items) *items = b->total;
    if (units) *units = b->nunits;
    if (grid) *grid = b->grid;
  });
}

void tqc_batch_destroy(tqc_batch_t batch) { delete reinterpret_cast<Batch *>(batch); }

tqc_status tqc_plan_autotune(tqc_plan_t plan, void *out, uint64_t out_bytes, int32_t reps, void *stream) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !out) fail(TQC_ERR_INVALID_ARG, "null argument");
    if (reps < 1) reps = 1;
    autotune_plan(p, out, out_bytes, reps, (hipStream_t)stream);
  });
}

tqc_status tqc_autotune_save(const char *path) {
  return guarded([&] {
    if (!path) fail(TQC_ERR_INVALID_ARG, "null path");
    FILE *f = fopen(path, "w");
    if (!f) fail(TQC_ERR_INVALID_ARG, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    fprintf(f, "# tqc autotune table: gfx950 hip-runtime %d\n# prec log2m log2n log2k tile ms\n", rt);
    for (auto &kv : g_tune)
      fprintf(f, "%d %d %d %d %d %.6f\n", kv.first.prec, kv.first.lm, kv.first.ln, kv.first.lk,
              kv.second.first, kv.second.second);
    fclose(f);
  });
}

tqc_status tqc_autotune_load(const char *path) {
  return guarded([&] {
    if (!path) fail(TQC_ERR_INVALID_ARG, "null path");
    FILE *f = fopen(path, "r");
    if (!f) fail(TQC_ERR_INVALID_ARG, "cannot read %s", path);
    char line[256];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    while (fgets(line, sizeof(line), f)) {
      if (line[0] == '#') continue;
      int pr, lm, ln, lk2, tile;
      double ms;
      if (sscanf(line, "%d %d %d %d %d %lf", &pr, &lm, &ln, &lk2, &tile, &ms) == 6 && tile >= 0 &&
          tile <= 2)
        g_tune[TuneKey{pr, lm, ln, lk2}] = {tile, ms};
    }
    fclose(f);
  });
}

struct tqc_costmodel_s : CostModel {};

tqc_status tqc_costmodel_create(uint64_t seed, tqc_costmodel_t *out) {
  return guarded([&] {
    if (!out) fail(TQC_ERR_INVALID_ARG, "null argument");
    *out = reinterpret_cast<tqc_costmodel_t>(create_costmodel(seed));
  });
}

void tqc_costmodel_destroy(tqc_costmodel_t m) { delete reinterpret_cast<CostModel *>(m); }

int32_t tqc_costmodel_num_params(void) { return kParams; }
int32_t tqc_costmodel_num_features(void) { return kFeat; }

tqc_status tqc_costmodel_get_params(tqc_costmodel_t mp, float *out, int32_t n) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !out || n < kParams) fail(TQC_ERR_INVALID_ARG, "bad argument");
    HIP_OK(hipMemcpy(out, m->d_theta, kParams * 4, hipMemcpyDeviceToHost));
  });
}

tqc_status tqc_costmodel_set_params(tqc_costmodel_t mp, const float *in, int32_t n) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !in || n < kParams) fail(TQC_ERR_INVALID_ARG, "bad argument");
    HIP_OK(hipMemcpy(m->d_theta, in, kParams * 4, hipMemcpyHostToDevice));
  });
}

tqc_status tqc_costmodel_forward(tqc_costmodel_t mp, const float *x, int64_t n, float *y, void *stream) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !x || !y || n < 1) fail(TQC_ERR_INVALID_ARG, "bad argument");
    costmodel_forward_raw(m, x, n, y, (hipStream_t)stream);
  });
}

tqc_status tqc_costmodel_gradients(tqc_costmodel_t mp, const float *x, const float *t, int64_t n,
                                   float *grad, void *stream) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !x || !t || !grad || n < 1) fail(TQC_ERR_INVALID_ARG, "bad argument");
    costmodel_grad_raw(m, x, t, n, grad, (hipStream_t)stream);
  });
}

tqc_status tqc_costmodel_train(tqc_costmodel_t mp, const float *feats, const float *seconds, int64_t n,
                               const tqc_train_options *opt, float *loss_per_epoch, void *stream) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !feats || !seconds) fail(TQC_ERR_INVALID_ARG, "bad argument");
    tqc_train_options o{};
    if (opt) o = *opt;
    costmodel_train(m, feats, seconds, n, o, loss_per_epoch, (hipStream_t)stream);
  });
}

tqc_status tqc_costmodel_predict(tqc_costmodel_t mp, const float *feats, int64_t n, double *seconds,
                                 void *stream) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !feats || !seconds || n < 1) fail(TQC_ERR_INVALID_ARG, "bad argument");
    costmodel_predict(m, feats, n, seconds, (hipStream_t)stream);
  });
}

tqc_status tqc_costmodel_save(tqc_costmodel_t mp, const char *path) {
  return guarded([&] {
    CostModel *m = reinterpret_cast<CostModel *>(mp);
    if (!m || !path) fail(TQC_ERR_INVALID_ARG, "bad argument");
    std::vector<float> th(kParams);
    HIP_OK(hipMemcpy(th.data(), m->d_theta, kParams * 4, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "w");
    if (!f) fail(TQC_ERR_INVALID_ARG, "cannot write %s", path);
    fprintf(f, "tqc-costmodel %d %d %d\n", kFeat, kHid, kParams);
    for (int i = 0; i < kFeat; ++i) fprintf(f, "%.9g %.9g\n", m->fmean[i], m->fstd[i]);
    fprintf(f, "%.9g %.9g\n", m->tmean, m->tstd);
    for (int i = 0; i < kParams; ++i) fprintf(f, "%.9g\n", th[i]);
    fclose(f);
  });
}

tqc_status tqc_costmodel_load(const char *path, tqc_costmodel_t *out) {
  return guarded([&] {
    if (!path || !out) fail(TQC_ERR_INVALID_ARG, "bad argument");
    FILE *f = fopen(path, "r");
    if (!f) fail(TQC_ERR_INVALID_ARG, "cannot read %s", path);
    int nf = 0, nh = 0, np = 0;
    if (fscanf(f, "tqc-costmodel %d %d %d", &nf, &nh, &np) != 3 || nf != kFeat || nh != kHid ||
        np != kParams) {
      fclose(f);
      fail(TQC_ERR_INVALID_ARG, "%s is not a cost model of this build", path);
    }
    std::unique_ptr<CostModel> m(create_costmodel(1));
    bool ok = true;
    for (int i = 0; i < kFeat; ++i) ok &= fscanf(f, "%f %f", &m->fmean[i], &m->fstd[i]) == 2;
    ok &= fscanf(f, "%f %f", &m->tmean, &m->tstd) == 2;
    std::vector<float> th(kParams);
    for (int i = 0; i < kParams; ++i) ok &= fscanf(f, "%f", &th[i]) == 1;
    fclose(f);
    if (!ok) fail(TQC_ERR_INVALID_ARG, "%s is truncated", path);
    HIP_OK(hipMemcpy(m->d_theta, th.data(), kParams * 4, hipMemcpyHostToDevice));
    *out = reinterpret_cast<tqc_costmodel_t>(m.release());
  });
}

tqc_status tqc_plan_step_features(tqc_plan_t plan, float *out, int32_t max_steps) {
  return guarded([&] {
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p || !out) fail(TQC_ERR_INVALID_ARG, "bad argument");
    if (max_steps < (int)p->steps.size()) fail(TQC_ERR_SHAPE, "need %zu rows", p->steps.size());
    for (size_t i = 0; i < p->steps.size(); ++i) {
      const Step &st = p->steps[i];
      StepShape sh{st.lm, st.ln, st.lk, st.kpad_log2, st.root ? 1 : 0,
                   p->nodes[st.out].slice_dep ? 1 : 0, st.tile};
      shape_features(sh, p->prec, p->out_dtype, p->num_slices, out + i * kFeat);
    }
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
