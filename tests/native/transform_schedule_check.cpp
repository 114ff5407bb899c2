// Host check of the separable Pauli transform schedule (transform_sched.hpp):
// emulates the pass kernel's index math on the CPU with bounds checks (every
// read inside the source layout, every destination entry written exactly
// once) and compares the result with the per-entry sums of the Sec. II-A
// maps over every combination of variants, on random tensors with 3..7 cuts.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <random>
#include "../../paper_2502_03445_amd/csrc/transform_sched.hpp"
namespace tqc {
[[noreturn]] void fail(tqc_status, const char *fmt, ...) { va_list ap; va_start(ap, fmt); vfprintf(stderr, fmt, ap); va_end(ap); abort(); }
}
using namespace tqc;
static void down_map(const double r[4], double p[4]) { double s01 = r[0] + r[1]; p[0] = s01; p[1] = 2.0 * r[2] - s01; p[2] = 2.0 * r[3] - s01; p[3] = r[0] - r[1]; }
static void up_map(const double v[6], double p[4]) { p[0] = v[0] + v[1]; p[1] = v[2] - v[3]; p[2] = v[4] - v[5]; p[3] = v[0] - v[1]; }
static void emulate(const TransformPassArgs &a, const std::vector<double> &in, std::vector<double> &out) {
  int NA = a.up[0] ? 6 : 4, NB = a.g == 2 ? (a.up[1] ? 6 : 4) : 1;
  std::vector<int> hits(out.size(), 0);
  for (uint64_t f = 0; f < a.nfree; ++f) {
    uint64_t r = f, ib = 0, ob = 0;
    for (int s = 0; s < a.nseg - 1; ++s) { uint64_t q = r / a.seg_ext[s], c = r - q * a.seg_ext[s]; ib += c * a.seg_in[s]; ob += c * a.seg_out[s]; r = q; }
    ib += r * a.seg_in[a.nseg - 1]; ob += r * a.seg_out[a.nseg - 1];
    double v[36];
    for (int ia = 0; ia < NA; ++ia) for (int jb = 0; jb < NB; ++jb) {
      uint64_t off = ib + (a.up[0] ? (uint64_t)(ia >> 1) * a.row_in[0] + (uint64_t)(ia & 1) * a.bit_in[0] : (uint64_t)ia * a.row_in[0]);
      if (a.g == 2) off += a.up[1] ? (uint64_t)(jb >> 1) * a.row_in[1] + (uint64_t)(jb & 1) * a.bit_in[1] : (uint64_t)jb * a.row_in[1];
      if (off >= in.size()) { printf("OOB read %llu >= %zu\n", (unsigned long long)off, in.size()); exit(1); }
      v[ia * NB + jb] = in[off];
    }
    double t[24];
    for (int jb = 0; jb < NB; ++jb) { double col[6], p[4]; for (int ia = 0; ia < NA; ++ia) col[ia] = v[ia * NB + jb]; if (a.up[0]) up_map(col, p); else down_map(col, p); for (int sa = 0; sa < 4; ++sa) t[sa * NB + jb] = p[sa]; }
    for (int sa = 0; sa < 4; ++sa) {
      if (a.g == 1) { uint64_t o = ob + sa * a.row_out[0]; if (o >= out.size()) { printf("OOB write\n"); exit(1); } out[o] = t[sa]; hits[o]++; }
      else { double p[4]; if (a.up[1]) up_map(t + sa * NB, p); else down_map(t + sa * NB, p);
        for (int sb = 0; sb < 4; ++sb) { uint64_t o = ob + sa * a.row_out[0] + sb * a.row_out[1]; if (o >= out.size()) { printf("OOB write\n"); exit(1); } out[o] = p[sb]; hits[o]++; } }
    }
  }
  for (size_t i = 0; i < hits.size(); ++i) if (hits[i] != 1) { printf("entry %zu written %d times\n", i, hits[i]); exit(1); }
}
// reference: per entry, the sum over every combination of options
static double ref_entry(const TensorIn &t, const std::vector<double> &raw, uint64_t e) {
  int c = t.cuts.size(), o = t.outputs.size(), u = t.u;
  uint64_t cols = 1ull << (o + u), x = e & ((1ull << o) - 1), row = e >> o;
  std::vector<uint64_t> w(c); uint64_t acc = 1; for (int i = c - 1; i >= 0; --i) { w[i] = acc; acc *= t.up[i] ? 3 : 4; }
  std::vector<int> bb(c); int bi = 0; for (int i = 0; i < c; ++i) bb[i] = t.up[i] ? bi++ : -1;
  // enumerate per-cut terms
  std::vector<std::vector<std::pair<double, std::pair<uint64_t, uint64_t>>>> terms(c);
  for (int i = 0; i < c; ++i) {
    int s = (row >> (2 * (c - 1 - i))) & 3;
    if (t.up[i]) { int meas = s == 3 ? 0 : s; terms[i].push_back({1.0, {meas * w[i], 0}}); terms[i].push_back({s == 0 ? 1.0 : -1.0, {meas * w[i], 1ull << bb[i]}}); }
    else if (s == 0) { terms[i] = {{1.0, {0, 0}}, {1.0, {w[i], 0}}}; }
    else if (s == 3) { terms[i] = {{1.0, {0, 0}}, {-1.0, {w[i], 0}}}; }
    else { terms[i] = {{2.0, {(uint64_t)(s + 1) * w[i], 0}}, {-1.0, {0, 0}}, {-1.0, {w[i], 0}}}; }
  }
  double sum = 0; std::vector<int> idx(c, 0);
  while (true) {
    double coef = 1; uint64_t rin = 0, b = 0;
    for (int i = 0; i < c; ++i) { coef *= terms[i][idx[i]].first; rin += terms[i][idx[i]].second.first; b |= terms[i][idx[i]].second.second; }
    sum += coef * raw[rin * cols + ((x << u) | b)];
    int i = c - 1; for (; i >= 0; --i) { if (++idx[i] < (int)terms[i].size()) break; idx[i] = 0; } if (i < 0) break;
  }
  return sum;
}
int main() {
  std::mt19937_64 rng(1);
  int ncase = 0;
  for (int trial = 0; trial < 300; ++trial) {
    TensorIn t;
    int c = 3 + rng() % 5, o = rng() % 6;
    if (trial % 50 == 0) o = 0;
    t.u = 0; t.d = 0;
    for (int i = 0; i < c; ++i) { t.cuts.push_back(i); int up = rng() % 2; t.up.push_back(up); if (up) t.u++; else t.d++; }
    for (int i = 0; i < o; ++i) t.outputs.push_back(i);
    uint64_t rows = 1; for (int i = 0; i < c; ++i) rows *= t.up[i] ? 3 : 4;
    uint64_t cols = 1ull << (o + t.u);
    if (rows * cols > (1u << 22)) continue;
    std::vector<double> raw(rows * cols); std::uniform_real_distribution<double> U(0, 1); for (auto &v : raw) v = U(rng);
    TransformSchedule sc = transform_schedule(t);
    std::vector<double> cur = raw;
    for (size_t p = 0; p < sc.passes.size(); ++p) { std::vector<double> nxt(sc.passes[p].out_entries, NAN); emulate(sc.passes[p], cur, nxt); cur.swap(nxt); }
    if (cur.size() != t.pauli_entries()) { printf("size mismatch\n"); return 1; }
    double maxerr = 0, maxv = 0;
    for (uint64_t e = 0; e < cur.size(); e += 1 + cur.size() / 4096) { double r = ref_entry(t, raw, e); maxerr = std::max(maxerr, std::fabs(r - cur[e])); maxv = std::max(maxv, std::fabs(r)); }
    if (maxerr > 1e-13 * std::max(1.0, maxv)) { printf("trial %d c %d o %d err %g\n", trial, c, o, maxerr); return 1; }
    ++ncase;
  }
  printf("ok %d cases\n", ncase);
}
