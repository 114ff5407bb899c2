// Cut search by greedy graph growing (Sec. VI, Alg. 2-3, Table I).
//
// The circuit DAG keeps one vertex per two-qubit gate and one edge per wire
// segment between consecutive two-qubit gates of a qubit.  Every vertex
// starts as its own partition; adjacent partitions are merged greedily by
// the merging cost of Table I until no merge is allowed.  Partition metrics:
// s = two-qubit gates; w = qubits, one per maximal run of a wire's
// two-qubit gates inside the partition (a wire that leaves and returns is a
// second qubit of the subcircuit); cuts(P) = edges with exactly one end in
// P; the contraction edges of neighbours P and Q are cuts(P) | cuts(Q)
// (internal and external edges, Sec. III-C).  The cost of merging P and Q
// (Alg. 3) is c(w_T; w_max) + c(s_T; s_max) + c(K_T; K_t) for the trial
// union T, K_T the largest contraction-edge count between T and one of its
// neighbours; c = x / T at or below the threshold, not allowed above it for
// w and s, 4^(x - T) + 1 above it for K.  Alg. 2 merges the cheapest pair
// with cost <= Q_max (ties: smaller first vertices) and then re-costs only
// the pairs that touch the merged partition.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <limits>
#include <map>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace tqc {

namespace {

struct Dag {
  std::vector<int> gate_of;                // vertex -> gate index
  std::vector<std::vector<int>> wire;      // qubit -> its vertices in order
  std::vector<std::array<int, 2>> edge;    // (earlier vertex, later vertex), sorted
};

double cost_of(int x, int thr, bool hard) {
  if (x <= thr) return double(x) / double(thr);
  if (hard || x - thr >= 512) return std::numeric_limits<double>::infinity();
  return std::ldexp(1.0, 2 * (x - thr)) + 1.0;
}

struct Grower {
  const Dag &g;
  int w_max, s_max, k_t;
  std::vector<int> label;                  // vertex -> partition
  std::map<int, std::vector<int>> members; // partition -> vertices (ascending)
  size_t words;

  Grower(const Dag &d, int w, int s, int k) : g(d), w_max(w), s_max(s), k_t(k) {
    const int nv = (int)g.gate_of.size();
    label.resize(nv);
    for (int v = 0; v < nv; ++v) {
      label[v] = v;
      members[v] = {v};
    }
    words = (g.edge.size() + 63) / 64;
  }

  // edges with exactly one end inside the vertex set flagged by `in`
  std::vector<uint64_t> cut_bits(const std::vector<char> &in) const {
    std::vector<uint64_t> b(words, 0);
    for (size_t e = 0; e < g.edge.size(); ++e)
      if (in[g.edge[e][0]] != in[g.edge[e][1]]) b[e >> 6] |= 1ull << (e & 63);
    return b;
  }

  std::vector<char> flags_of(int p, int q = -1) const {
    std::vector<char> in(label.size(), 0);
    for (int v : members.at(p)) in[v] = 1;
    if (q >= 0)
      for (int v : members.at(q)) in[v] = 1;
    return in;
  }

  int width(const std::vector<char> &in) const {
    int runs = 0;
    for (const auto &vs : g.wire) {
      bool inside = false;
      for (int v : vs) {
        if (in[v] && !inside) ++runs;
        inside = in[v] != 0;
      }
    }
    return runs;
  }

  double trial_cost(int p, int q) const {
    const std::vector<char> in = flags_of(p, q);
    const int w = width(in);
    const int s = (int)(members.at(p).size() + members.at(q).size());
    const std::vector<uint64_t> tc = cut_bits(in);
    // neighbours of the union
    std::vector<int> nb;
    for (size_t e = 0; e < g.edge.size(); ++e) {
      const int a = g.edge[e][0], b = g.edge[e][1];
      if (in[a] != in[b]) nb.push_back(in[a] ? label[b] : label[a]);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    int k = 0;
    for (int r : nb) {
      const std::vector<uint64_t> rc = cut_bits(flags_of(r));
      int cnt = 0;
      for (size_t i = 0; i < words; ++i) cnt += __builtin_popcountll(tc[i] | rc[i]);
      k = std::max(k, cnt);
    }
    return cost_of(w, w_max, true) + cost_of(s, s_max, true) + cost_of(k, k_t, false);
  }

  std::vector<std::pair<int, int>> live_pairs() const {
    std::vector<std::pair<int, int>> ps;
    for (const auto &e : g.edge) {
      const int a = label[e[0]], b = label[e[1]];
      if (a != b) ps.push_back({std::min(a, b), std::max(a, b)});
    }
    std::sort(ps.begin(), ps.end());
    ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
    return ps;
  }

  void run(double q_max) {
    std::map<std::pair<int, int>, double> cost;
    for (const auto &pq : live_pairs()) cost[pq] = trial_cost(pq.first, pq.second);
    for (;;) {
      const auto live = live_pairs();
      bool found = false;
      double bc = 0;
      int bf0 = 0, bf1 = 0;
      std::pair<int, int> best;
      for (const auto &pq : live) {
        const double c = cost.at(pq);
        if (!(c <= q_max)) continue;
        int f0 = members.at(pq.first).front(), f1 = members.at(pq.second).front();
        if (f0 > f1) std::swap(f0, f1);
        if (!found || c < bc || (c == bc && (f0 < bf0 || (f0 == bf0 && f1 < bf1)))) {
          found = true;
          bc = c;
          bf0 = f0;
          bf1 = f1;
          best = pq;
        }
      }
      if (!found) break;
      const int p = best.first, q = best.second;
      std::vector<int> &mp = members[p];
      const std::vector<int> mq = members[q];
      members.erase(q);
      mp.insert(mp.end(), mq.begin(), mq.end());
      std::sort(mp.begin(), mp.end());
      for (int v : mp) label[v] = p;
      const auto now = live_pairs();
      std::map<std::pair<int, int>, double> next;
      for (const auto &pq : now) {
        auto it = cost.find(pq);
        if (pq.first == p || pq.second == p || it == cost.end()) next[pq] = trial_cost(pq.first, pq.second);
        else next[pq] = it->second;
      }
      cost.swap(next);
    }
  }
};

}  // namespace

int find_cuts(int num_qubits, int num_gates, const int32_t *gq, int w_max, int s_max, int k_t, double q_max,
              int32_t *labels) {
  Dag g;
  g.wire.assign(num_qubits, {});
  std::vector<int> vid(num_gates, -1);
  std::vector<int> last(num_qubits, -1);
  for (int i = 0; i < num_gates; ++i) {
    const int a = gq[2 * i], b = gq[2 * i + 1];
    if (a < 0 || a >= num_qubits || b >= num_qubits || b == a)
      fail(TQC_ERR_INVALID_ARG, "gate %d acts on qubits (%d, %d)", i, a, b);
    if (b < 0) continue;
    const int v = (int)g.gate_of.size();
    g.gate_of.push_back(i);
    vid[i] = v;
    for (int q : {a, b}) {
      if (last[q] >= 0) g.edge.push_back({last[q], v});
      last[q] = v;
      g.wire[q].push_back(v);
    }
  }
  std::sort(g.edge.begin(), g.edge.end());
  Grower gr(g, w_max, s_max, k_t);
  gr.run(q_max);
  // labels in order of each partition's first vertex
  std::vector<std::pair<int, int>> firsts;
  for (const auto &kv : gr.members) firsts.push_back({kv.second.front(), kv.first});
  std::sort(firsts.begin(), firsts.end());
  std::map<int, int> ren;
  for (size_t i = 0; i < firsts.size(); ++i) ren[firsts[i].second] = (int)i;
  for (int i = 0; i < num_gates; ++i) labels[i] = vid[i] >= 0 ? ren[gr.label[vid[i]]] : -1;
  return (int)firsts.size();
}

}  // namespace tqc
