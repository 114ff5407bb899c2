// Contraction planning: order (Sec. III-E1), slicing (Sec. III-E2) and the
// mapping of each pairwise contraction onto a plain GEMM.
//
// Cost of one step joining tensor sets S1 and S2 (Sec. III-C): the shared
// cut indices form K = 4^shared, the remaining indices of each side form
// M and N (4 per open cut, 2 per free output qubit), and the step costs
// M*N*K multiply-adds.  The planner prices a step as
//     max(2*M*N*K / mfma_peak, bytes / hbm_bandwidth) + launch overhead,
// a roofline refinement of Eq. (7) (the paper notes that plain flops over
// peak overestimates GPU time).  Exact dynamic programming over subsets
// finds the cheapest binary tree for up to 13 tensors; beyond that, a
// greedy (or randomised greedy) pair selection is used.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <iterator>
#include <limits>
#include <memory>
#include <numeric>
#include <random>

#include "internal.hpp"
#include "transform_sched.hpp"

namespace tqc {

double prec_peak_flops(Prec p) {
  switch (p) {
    case Prec::F64: return 78.6e12;
    case Prec::F32: return 157.3e12;
    case Prec::BF16X3: return 2.5e15 / 3.0;
    case Prec::BF16X6: return 2.5e15 / 6.0;
    case Prec::F16X3: return 2.5e15 / 3.0;
  }
  return 157.3e12;
}
int prec_bytes(Prec p) {
  switch (p) {
    case Prec::F64: return 8;
    case Prec::F32: return 4;
    case Prec::BF16X3: return 4;
    case Prec::BF16X6: return 6;
    case Prec::F16X3: return 4;
  }
  return 4;
}
static int prec_kmin_log2(Prec p) {
  // smallest operand row stride: one MFMA k-group per lane group
  return (p == Prec::BF16X3 || p == Prec::BF16X6 || p == Prec::F16X3) ? 5 : 4;
}
static int prec_planes(Prec p) {
  return p == Prec::BF16X3 ? 2 : (p == Prec::BF16X6 ? 3 : 1);
}
static int plane_elem_bytes(Prec p) {
  // float16-split plans keep their operands and intermediates in float32
  return p == Prec::F64 ? 8 : ((p == Prec::F32 || p == Prec::F16X3) ? 4 : 2);
}

static constexpr double kHbmBw = 8.0e12;
static constexpr double kLaunch = 4.0e-6;

namespace {

struct Structure {
  int m = 0, K = 0;
  std::vector<uint64_t> cutmask;   // per leaf: unsliced cuts touching it
  std::vector<int> qubits;         // per leaf: free output qubits
  std::vector<uint64_t> endpoint_a, endpoint_b;  // per cut: leaf bitmask (single bit)
  uint64_t sliced_mask = 0;
  std::vector<int> leaf_slice_dep;
};

Structure make_structure(const Network &net, const std::vector<int> &sliced,
                         const std::vector<int> &fixed_q) {
  Structure s;
  s.m = net.m;
  s.K = net.K;
  for (int c : sliced) s.sliced_mask |= (1ull << c);
  s.cutmask.assign(net.m, 0);
  s.qubits.assign(net.m, 0);
  s.leaf_slice_dep.assign(net.m, 0);
  for (int j = 0; j < net.m; ++j) {
    for (int c : net.t[j].cuts) {
      if (s.sliced_mask >> c & 1) s.leaf_slice_dep[j] = 1;
      else s.cutmask[j] |= (1ull << c);
    }
    int q = 0;
    for (int o : net.t[j].outputs)
      if (std::find(fixed_q.begin(), fixed_q.end(), o) == fixed_q.end()) ++q;
    s.qubits[j] = q;
  }
  return s;
}

struct StepCost {
  int lm, ln, lk;
  double time, flops, bytes;
};

// open cuts of a leaf set = cuts with exactly one endpoint in the set
inline uint64_t open_cuts(const std::vector<uint64_t> &leaf_cutmask, uint64_t set) {
  uint64_t x = 0;
  for (uint64_t s = set; s; s &= s - 1) x ^= leaf_cutmask[__builtin_ctzll(s)];
  return x;
}

StepCost step_cost(Prec prec, tqc_dtype out_dtype, uint64_t open1, int q1, uint64_t open2, int q2,
                   bool root, uint64_t slices, bool slice_dep) {
  uint64_t shared = open1 & open2;
  StepCost c;
  c.lk = 2 * __builtin_popcountll(shared);
  c.lm = 2 * __builtin_popcountll(open1 & ~shared) + q1;
  c.ln = 2 * __builtin_popcountll(open2 & ~shared) + q2;
  double M = std::ldexp(1.0, c.lm), N = std::ldexp(1.0, c.ln), K = std::ldexp(1.0, c.lk);
  double Kp = std::max(K, std::ldexp(1.0, prec_kmin_log2(prec)));
  c.flops = 2.0 * M * N * K;
  double eb = prec_bytes(prec);
  double out_b;
  if (root) {
    if (slices > 1) out_b = 16.0;  // float64 read-modify-write per slice
    else out_b = out_dtype == TQC_F64 ? 8.0 : 4.0;
  } else {
    out_b = eb;
  }
  c.bytes = eb * (M * Kp + N * Kp) + out_b * M * N;
  c.time = std::max(c.flops / prec_peak_flops(prec), c.bytes / kHbmBw) + kLaunch;
  if (slice_dep) {
    c.time *= double(slices);
    c.flops *= double(slices);
    c.bytes *= double(slices);
  }
  return c;
}

// ---- exact DP over subsets
std::vector<int> dp_order(const Structure &s, Prec prec, tqc_dtype out_dtype, uint64_t slices) {
  const int m = s.m;
  const uint64_t full = (m == 64) ? ~0ull : ((1ull << m) - 1);
  const size_t NS = size_t(1) << m;
  std::vector<double> best(NS, std::numeric_limits<double>::infinity());
  std::vector<uint32_t> split(NS, 0);
  std::vector<uint64_t> openm(NS, 0);
  std::vector<int> qsum(NS, 0);
  std::vector<uint8_t> dep(NS, 0);
  for (size_t S = 1; S < NS; ++S) {
    int j = __builtin_ctzll(S);
    size_t rest = S & (S - 1);
    openm[S] = openm[rest] ^ s.cutmask[j];
    qsum[S] = qsum[rest] + s.qubits[j];
    dep[S] = dep[rest] | (uint8_t)s.leaf_slice_dep[j];
  }
  for (int j = 0; j < m; ++j) best[size_t(1) << j] = 0.0;
  // increasing popcount order is implied by numeric order for subsets of S
  for (size_t S = 1; S < NS; ++S) {
    if ((S & (S - 1)) == 0) continue;
    size_t low = S & (~S + 1);
    bool root = (S == full);
    for (size_t S1 = (S - 1) & S; S1; S1 = (S1 - 1) & S) {
      if (!(S1 & low)) continue;
      size_t S2 = S ^ S1;
      double b = best[S1] + best[S2];
      if (b >= best[S]) continue;
      StepCost c = step_cost(prec, out_dtype, openm[S1], qsum[S1], openm[S2], qsum[S2], root,
                             slices, dep[S] != 0);
      if (b + c.time < best[S]) {
        best[S] = b + c.time;
        split[S] = (uint32_t)S1;
      }
    }
  }
  // emit SSA order by post-order traversal of the split tree
  std::vector<int> order;
  int next_id = m;
  std::function<int(size_t)> emit = [&](size_t S) -> int {
    if ((S & (S - 1)) == 0) return __builtin_ctzll(S);
    int a = emit(split[S]);
    int b = emit(S ^ split[S]);
    order.push_back(a);
    order.push_back(b);
    return next_id++;
  };
  emit(full);
  return order;
}

// ---- greedy / randomised greedy
std::vector<int> greedy_order(const Structure &s, Prec prec, tqc_dtype out_dtype, uint64_t slices,
                              std::mt19937_64 *rng, double temperature) {
  const int m = s.m;
  std::vector<uint64_t> sets;   // leaf-bitmask per live id (only up to 64 leaves)
  std::vector<int> ids;
  for (int j = 0; j < m; ++j) {
    sets.push_back(1ull << j);
    ids.push_back(j);
  }
  std::vector<uint64_t> open(m), dep(m);
  std::vector<int> q(m);
  for (int j = 0; j < m; ++j) {
    open[j] = s.cutmask[j];
    q[j] = s.qubits[j];
    dep[j] = s.leaf_slice_dep[j];
  }
  std::vector<int> order;
  int next = m;
  while (ids.size() > 1) {
    struct Cand { size_t i, j; double t; };
    std::vector<Cand> cands;
    bool any_shared = false;
    for (size_t i = 0; i < ids.size(); ++i)
      for (size_t j = i + 1; j < ids.size(); ++j)
        if (open[i] & open[j]) any_shared = true;
    for (size_t i = 0; i < ids.size(); ++i)
      for (size_t j = i + 1; j < ids.size(); ++j) {
        if (any_shared && !(open[i] & open[j])) continue;
        bool root = ids.size() == 2;
        StepCost c = step_cost(prec, out_dtype, open[i], q[i], open[j], q[j], root, slices,
                               dep[i] || dep[j]);
        // greedy score: step time, minus a small credit for shrinking tensors
        cands.push_back({i, j, c.time});
      }
    size_t pick = 0;
    double tmin = cands[0].t;
    for (size_t c = 1; c < cands.size(); ++c)
      if (cands[c].t < tmin) { tmin = cands[c].t; pick = c; }
    if (rng && temperature > 0) {
      std::vector<double> w(cands.size());
      for (size_t c = 0; c < cands.size(); ++c)
        w[c] = std::exp(-(std::log(cands[c].t) - std::log(tmin)) / temperature);
      std::discrete_distribution<size_t> dist(w.begin(), w.end());
      pick = dist(*rng);
    }
    size_t i = cands[pick].i, j = cands[pick].j;
    order.push_back(ids[i]);
    order.push_back(ids[j]);
    uint64_t no = open[i] ^ open[j];
    int nq = q[i] + q[j];
    uint64_t nd = dep[i] | dep[j];
    // remove j then i (j > i)
    for (size_t k : {j, i}) {
      ids.erase(ids.begin() + k);
      open.erase(open.begin() + k);
      q.erase(q.begin() + k);
      dep.erase(dep.begin() + k);
    }
    ids.push_back(next++);
    open.push_back(no);
    q.push_back(nq);
    dep.push_back(nd);
  }
  return order;
}

}  // namespace

// ---------------------------------------------------------- plan assembly
static void assemble(Plan &p) {
  Network &net = *p.net;
  const int m = net.m, K = net.K;
  p.nodes.assign(m + std::max(0, m - 1), Node{});
  p.steps.assign(std::max(0, m - 1), Step{});
  uint64_t sliced_mask = 0;
  for (int c : p.sliced) sliced_mask |= 1ull << c;
  // label sets
  std::vector<std::vector<int>> lab(p.nodes.size());
  for (int j = 0; j < m; ++j) {
    auto &L = lab[j];
    for (int c : net.t[j].cuts)
      if (!(sliced_mask >> c & 1)) {
        L.push_back(cut_label(c, 0));
        L.push_back(cut_label(c, 1));
      }
    for (int o : net.t[j].outputs)
      if (std::find(p.fixed_q.begin(), p.fixed_q.end(), o) == p.fixed_q.end())
        L.push_back(2 * K + o);
    std::sort(L.begin(), L.end());
    p.nodes[j].leaf = j;
    for (int c : net.t[j].cuts)
      if (sliced_mask >> c & 1) p.nodes[j].slice_dep = true;
  }
  std::vector<int> used(p.nodes.size(), 0);
  for (int s = 0; s < m - 1; ++s) {
    int a = p.order[2 * s], b = p.order[2 * s + 1];
    if (a < 0 || b < 0 || a >= m + s || b >= m + s || a == b || used[a] || used[b])
      fail(TQC_ERR_INVALID_ARG, "contraction order: step %d joins ids %d and %d, which are not "
           "two distinct live tensors", s, a, b);
    used[a] = used[b] = 1;
    Step &st = p.steps[s];
    st.a = a;
    st.b = b;
    st.out = m + s;
    std::vector<int> &La = lab[a], &Lb = lab[b];
    std::set_intersection(La.begin(), La.end(), Lb.begin(), Lb.end(), std::back_inserter(st.k_labels));
    std::set_difference(La.begin(), La.end(), Lb.begin(), Lb.end(), std::back_inserter(st.m_labels));
    std::set_difference(Lb.begin(), Lb.end(), La.begin(), La.end(), std::back_inserter(st.n_labels));
    std::vector<int> &Lo = lab[m + s];
    std::set_union(st.m_labels.begin(), st.m_labels.end(), st.n_labels.begin(), st.n_labels.end(),
                   std::back_inserter(Lo));
    std::sort(Lo.begin(), Lo.end());
    p.nodes[m + s].producer = s;
    p.nodes[m + s].slice_dep = p.nodes[a].slice_dep || p.nodes[b].slice_dep;
    st.lm = (int)st.m_labels.size();
    st.ln = (int)st.n_labels.size();
    st.lk = (int)st.k_labels.size();
    // cuts involved (Sec. III-C: shared plus open cut indices of the pair)
    std::vector<int> cu;
    for (int l : La) if (l < 2 * K) cu.push_back(l / 2);
    for (int l : Lb) if (l < 2 * K) cu.push_back(l / 2);
    std::sort(cu.begin(), cu.end());
    cu.erase(std::unique(cu.begin(), cu.end()), cu.end());
    st.cuts_involved = (int)cu.size();
  }
  const int root = (m == 1) ? 0 : (2 * m - 2);
  // root layout: free qubits ascending
  p.out_labels.clear();
  for (int q = 0; q < net.n; ++q)
    if (std::find(p.fixed_q.begin(), p.fixed_q.end(), q) == p.fixed_q.end())
      p.out_labels.push_back(2 * K + q);
  p.out_bits = (int)p.out_labels.size();
  {
    std::vector<int> rl = lab[root];
    std::vector<int> ol = p.out_labels;
    std::sort(ol.begin(), ol.end());
    if (rl != ol) fail(TQC_ERR_INTERNAL, "root tensor labels do not match the free qubits");
  }
  p.nodes[root].labels = p.out_labels;
  p.nodes[root].kpad_log2 = 0;
  p.nodes[root].log2k = 0;
  // top-down layouts
  const int kmin = prec_kmin_log2(p.prec);
  for (int s = m - 2; s >= 0; --s) {
    Step &st = p.steps[s];
    Node &on = p.nodes[st.out];
    st.root = (st.out == root);
    // position of each label in the output node's storage
    auto pos_of = [&](int l) -> int {
      auto it = std::find(on.labels.begin(), on.labels.end(), l);
      if (it == on.labels.end()) fail(TQC_ERR_INTERNAL, "label missing from layout");
      int i = int(it - on.labels.begin());
      return i < on.log2k ? i : (i - on.log2k + on.kpad_log2);
    };
    auto by_pos = [&](std::vector<int> &v) {
      std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return pos_of(x) < pos_of(y); });
    };
    by_pos(st.m_labels);
    by_pos(st.n_labels);
    st.posM.clear();
    st.posN.clear();
    for (int l : st.m_labels) st.posM.push_back(pos_of(l));
    for (int l : st.n_labels) st.posN.push_back(pos_of(l));
    st.kpad_log2 = std::max(st.lk, kmin);
    for (int side = 0; side < 2; ++side) {
      Node &nd = p.nodes[side == 0 ? st.a : st.b];
      nd.labels = st.k_labels;
      const auto &rest = side == 0 ? st.m_labels : st.n_labels;
      nd.labels.insert(nd.labels.end(), rest.begin(), rest.end());
      nd.log2k = st.lk;
      nd.kpad_log2 = st.kpad_log2;
    }
  }
  // sizes, planes, workspace offsets
  uint64_t off = 0;
  auto align = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  // float64 Pauli tensors of raw inputs (transform output)
  for (int j = 0; j < m; ++j)
    if (net.t[j].basis == TQC_BASIS_RAW) off = align(off + net.t[j].pauli_entries() * 8);
  // ping-pong buffers of the multi-pass transform, one pair per tensor
  p.tscr_off.assign(m, 0);
  p.tscr_bytes.assign(m, 0);
  for (int j = 0; j < m; ++j)
    if (net.t[j].basis == TQC_BASIS_RAW && (int)net.t[j].cuts.size() >= kPassMinCuts) {
      p.tscr_bytes[j] = align(transform_schedule(net.t[j]).max_intermediate * 8);
      p.tscr_off[j] = off;
      off += 2 * p.tscr_bytes[j];
    }
  // split-K partial sums: the most any step may use on a 256-CU device with
  // its largest (128x128) tile, the case with the fewest tiles
  uint64_t pk = 0;
  for (const Step &st : p.steps) {
    if (st.kpad_log2 < 9) continue;
    const uint64_t M = 1ull << st.lm, N = 1ull << st.ln;
    const uint64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
    if (tiles >= 256) continue;
    int ks = 0;
    while ((tiles << ks) < 512 && ks < st.kpad_log2 - 8) ++ks;
    pk = std::max(pk, (M * N << ks) * 8);
  }
  p.splitk_bytes = align(pk);
  p.splitk_off = off;
  off += p.splitk_bytes;
  for (size_t i = 0; i < p.nodes.size(); ++i) {
    Node &nd = p.nodes[i];
    nd.rows = 1ull << (nd.labels.size() - nd.log2k);
    if ((int)i == root) {
      nd.planes = 1;
      nd.plane_bytes = 0;  // written to the caller's buffer
      continue;
    }
    nd.planes = prec_planes(p.prec);
    nd.plane_bytes = align(nd.elems() * plane_elem_bytes(p.prec));
    nd.offset = off;
    off += nd.plane_bytes * nd.planes;
  }
  // float16-split plans: the pairwise steps run in float32 (planes as
  // above); the final step's operands are split again into two float16
  // planes each
  if (p.prec == Prec::F16X3)
    for (const Step &st : p.steps)
      if (st.root)
        for (int i = 0; i < 2; ++i) {
          const Node &nd = p.nodes[i == 0 ? st.a : st.b];
          p.h16_plane[i] = align(nd.elems() * 2);
          p.h16_off[i] = off;
          off += 2 * p.h16_plane[i];
        }
  p.ws_bytes = off;
}

static void compute_stats(Plan &p) {
  tqc_plan_stats &s = p.stats;
  Network &net = *p.net;
  s.num_steps = (int)p.steps.size();
  s.num_sliced = (int)p.sliced.size();
  s.num_slices = p.num_slices;
  s.out_qubits = p.out_bits;
  s.out_entries = 1ull << p.out_bits;
  s.k_max_cuts = 0;
  s.flops = s.bytes = s.mults_per_state = s.predicted_seconds = 0;
  for (Step &st : p.steps) {
    bool dep = p.nodes[st.out].slice_dep;
    uint64_t open_a = 0, open_b = 0;
    (void)open_a; (void)open_b;
    double M = std::ldexp(1.0, st.lm), N = std::ldexp(1.0, st.ln), Kd = std::ldexp(1.0, st.lk);
    double Kp = std::ldexp(1.0, st.kpad_log2);
    double eb = prec_bytes(p.prec);
    double out_b = st.root ? (p.num_slices > 1 ? 16.0 : (p.out_dtype == TQC_F64 ? 8.0 : 4.0)) : eb;
    st.flops = 2.0 * M * N * Kd;
    st.bytes = eb * (M * Kp + N * Kp) + out_b * M * N;
    double mult = dep ? double(p.num_slices) : 1.0;
    double t = std::max(st.flops / prec_peak_flops(p.prec), st.bytes / kHbmBw) + kLaunch;
    s.flops += st.flops * mult;
    s.bytes += st.bytes * mult;
    s.predicted_seconds += t * mult;
    s.mults_per_state += std::ldexp(1.0, 2 * st.cuts_involved) * mult;
    s.k_max_cuts = std::max(s.k_max_cuts, st.cuts_involved);
  }
  uint64_t acc = 0;
  if (p.num_slices > 1 && p.out_dtype == TQC_F32) acc = (1ull << p.out_bits) * 8;
  s.workspace_bytes = p.ws_bytes + acc;
  (void)net;
}

static double plan_seconds_for(Network *net, Prec prec, tqc_dtype out, const std::vector<int> &sliced,
                               const std::vector<int> &fixed_q, const std::vector<int> &order) {
  Structure st = make_structure(*net, sliced, fixed_q);
  uint64_t slices = 1ull << (2 * sliced.size());
  // replay order
  std::vector<uint64_t> open(net->m + net->m), dep(2 * net->m);
  std::vector<int> q(2 * net->m);
  for (int j = 0; j < net->m; ++j) {
    open[j] = st.cutmask[j];
    q[j] = st.qubits[j];
    dep[j] = st.leaf_slice_dep[j];
  }
  double total = 0;
  for (int s = 0; s + 1 < net->m; ++s) {
    int a = order[2 * s], b = order[2 * s + 1];
    bool root = (s == net->m - 2);
    StepCost c = step_cost(prec, out, open[a], q[a], open[b], q[b], root, slices, dep[a] || dep[b]);
    total += c.time;
    open[net->m + s] = open[a] ^ open[b];
    q[net->m + s] = q[a] + q[b];
    dep[net->m + s] = dep[a] | dep[b];
  }
  return total;
}

std::vector<int> choose_order(Network *net, Prec prec, tqc_dtype out, const std::vector<int> &sliced,
                              const std::vector<int> &fixed_q) {
  Structure st = make_structure(*net, sliced, fixed_q);
  uint64_t slices = 1ull << (2 * sliced.size());
  if (net->m <= 1) return {};
  if (net->m <= 13) return dp_order(st, prec, out, slices);
  return greedy_order(st, prec, out, slices, nullptr, 0.0);
}

int default_tile(int lm, int ln) {
  const int lmn = std::min(lm, ln);
  if (lmn >= 7) return 0;
  if (lmn >= 6) return 1;
  return 2;
}

int kmin_log2(Prec p) { return prec_kmin_log2(p); }

std::vector<StepShape> order_shapes(Network *net, Prec prec, const std::vector<int> &sliced,
                                    const std::vector<int> &fixed_q, const std::vector<int> &order) {
  Structure st = make_structure(*net, sliced, fixed_q);
  const int m = net->m;
  std::vector<uint64_t> open(2 * m), dep(2 * m);
  std::vector<int> q(2 * m);
  for (int j = 0; j < m; ++j) {
    open[j] = st.cutmask[j];
    q[j] = st.qubits[j];
    dep[j] = st.leaf_slice_dep[j];
  }
  std::vector<StepShape> res;
  for (int s = 0; s + 1 < m; ++s) {
    const int a = order[2 * s], b = order[2 * s + 1];
    const uint64_t shared = open[a] & open[b];
    StepShape sh{};
    sh.lk = 2 * __builtin_popcountll(shared);
    sh.lm = 2 * __builtin_popcountll(open[a] & ~shared) + q[a];
    sh.ln = 2 * __builtin_popcountll(open[b] & ~shared) + q[b];
    sh.kpad = std::max(sh.lk, prec_kmin_log2(prec));
    sh.root = (s == m - 2);
    sh.slice_dep = (dep[a] || dep[b]) ? 1 : 0;
    sh.tile = default_tile(sh.lm, sh.ln);
    res.push_back(sh);
    open[m + s] = open[a] ^ open[b];
    q[m + s] = q[a] + q[b];
    dep[m + s] = dep[a] | dep[b];
  }
  return res;
}

std::vector<std::vector<int>> sample_orders(Network *net, Prec prec, tqc_dtype out,
                                            const std::vector<int> &sliced,
                                            const std::vector<int> &fixed_q, int count, uint64_t seed) {
  std::vector<std::vector<int>> res;
  if (net->m <= 1) return {std::vector<int>()};
  Structure st = make_structure(*net, sliced, fixed_q);
  const uint64_t slices = 1ull << (2 * sliced.size());
  res.push_back(choose_order(net, prec, out, sliced, fixed_q));
  res.push_back(greedy_order(st, prec, out, slices, nullptr, 0.0));
  std::mt19937_64 rng(seed ? seed : 0x9e3779b97f4a7c15ull);
  const double temps[4] = {0.3, 1.0, 3.0, 10.0};
  for (int i = 2; i < count; ++i) res.push_back(greedy_order(st, prec, out, slices, &rng, temps[i % 4]));
  return res;
}

// memory of a plan: workspace plus float64 accumulator
static uint64_t plan_memory(Plan &p) {
  uint64_t acc = (p.num_slices > 1 && p.out_dtype == TQC_F32) ? (1ull << p.out_bits) * 8 : 0;
  return p.ws_bytes + acc;
}

Plan *build_plan(Network *net, const tqc_plan_options &opt) {
  auto t0 = std::chrono::steady_clock::now();
  if (net->K > 64) fail(TQC_ERR_UNSUPPORTED, "more than 64 cuts");
  if (net->m > 64) fail(TQC_ERR_UNSUPPORTED, "more than 64 tensors");
  std::unique_ptr<Plan> p(new Plan());
  p->net = net;
  p->prec = Prec(int(opt.precision));
  if (int(opt.precision) < 0 || int(opt.precision) > 4) fail(TQC_ERR_INVALID_ARG, "precision");
  if (opt.out_dtype != TQC_F32 && opt.out_dtype != TQC_F64) fail(TQC_ERR_INVALID_ARG, "out_dtype");
  p->out_dtype = opt.out_dtype;
  if (opt.tile_policy < 0 || opt.tile_policy > 2) fail(TQC_ERR_INVALID_ARG, "tile_policy %d", opt.tile_policy);
  p->tile_policy = opt.tile_policy;
  if (opt.num_fixed < 0 || (opt.num_fixed > 0 && (!opt.fixed_qubits || !opt.fixed_values)))
    fail(TQC_ERR_INVALID_ARG, "fixed qubits");
  for (int i = 0; i < opt.num_fixed; ++i) {
    int q = opt.fixed_qubits[i], v = opt.fixed_values[i];
    if (q < 0 || q >= net->n) fail(TQC_ERR_INVALID_ARG, "fixed qubit %d out of range", q);
    if (v != 0 && v != 1) fail(TQC_ERR_INVALID_ARG, "fixed value of qubit %d is %d", q, v);
    if (std::find(p->fixed_q.begin(), p->fixed_q.end(), q) != p->fixed_q.end())
      fail(TQC_ERR_INVALID_ARG, "qubit %d fixed twice", q);
    p->fixed_q.push_back(q);
    p->fixed_v.push_back(v);
  }
  if (net->n - opt.num_fixed > 40) fail(TQC_ERR_UNSUPPORTED, "more than 2^40 output entries");
  const bool explicit_order = opt.num_order_steps > 0;
  if (explicit_order) {
    if (opt.num_order_steps != net->m - 1 || !opt.order)
      fail(TQC_ERR_INVALID_ARG, "order must have m-1 = %d steps", net->m - 1);
  }
  auto order_for = [&](const std::vector<int> &sl) {
    if (explicit_order) return std::vector<int>(opt.order, opt.order + 2 * opt.num_order_steps);
    return choose_order(net, p->prec, p->out_dtype, sl, p->fixed_q);
  };
  auto realize = [&](const std::vector<int> &sl) {
    p->sliced = sl;
    p->num_slices = 1ull << (2 * sl.size());
    p->order = order_for(sl);
    assemble(*p);
    compute_stats(*p);
  };
  if (opt.num_sliced >= 0) {
    std::vector<int> sl;
    if (opt.num_sliced > 0 && !opt.sliced_cuts) fail(TQC_ERR_INVALID_ARG, "sliced_cuts");
    for (int i = 0; i < opt.num_sliced; ++i) {
      int c = opt.sliced_cuts[i];
      if (c < 0 || c >= net->K) fail(TQC_ERR_INVALID_ARG, "sliced cut %d out of range", c);
      if (std::find(sl.begin(), sl.end(), c) != sl.end()) fail(TQC_ERR_INVALID_ARG, "cut sliced twice");
      sl.push_back(c);
    }
    if (sl.size() > 20) fail(TQC_ERR_UNSUPPORTED, "more than 20 sliced cuts");
    realize(sl);
    if (opt.mem_budget_bytes && plan_memory(*p) > opt.mem_budget_bytes)
      fail(TQC_ERR_PLAN_INFEASIBLE, "plan needs %llu bytes, budget %llu",
           (unsigned long long)plan_memory(*p), (unsigned long long)opt.mem_budget_bytes);
  } else {
    // Two-level slicing: slice the cut that shrinks the plan's memory most
    // (ties: lower predicted time, then lower cut id) until the packed inputs
    // and then the intermediates fit in the budget.
    std::vector<int> sl;
    realize(sl);
    while (opt.mem_budget_bytes && plan_memory(*p) > opt.mem_budget_bytes) {
      int best_c = -1;
      uint64_t best_mem = plan_memory(*p);
      double best_t = 0;
      for (int c = 0; c < net->K; ++c) {
        if (std::find(sl.begin(), sl.end(), c) != sl.end()) continue;
        std::vector<int> s2 = sl;
        s2.push_back(c);
        realize(s2);
        uint64_t mem = plan_memory(*p);
        double t = p->stats.predicted_seconds;
        if (mem < best_mem || (best_c >= 0 && mem == best_mem && t < best_t)) {
          best_c = c;
          best_mem = mem;
          best_t = t;
        }
      }
      if (best_c < 0 || sl.size() >= 20) {
        realize(sl);
        fail(TQC_ERR_PLAN_INFEASIBLE, "no slicing fits %llu bytes (best %llu)",
             (unsigned long long)opt.mem_budget_bytes, (unsigned long long)plan_memory(*p));
      }
      sl.push_back(best_c);
      realize(sl);
    }
  }
  (void)plan_seconds_for;
  auto t1 = std::chrono::steady_clock::now();
  p->stats.plan_seconds = std::chrono::duration<double>(t1 - t0).count();
  return p.release();
}

}  // namespace tqc
