// Host-side schedule of the separable Pauli transform of one raw tensor
// (Sec. II-A): the passes that turn its cuts into Pauli digits one or two at
// a time, with the strides of every index in the layouts before and after
// each pass.
//
// Raw layout: rows are mixed-radix digits over the tensor's cuts (first cut
// slowest; radix 3 = measurement basis at an upstream end, radix 4 =
// preparation at a downstream end); columns are x * 2^u + b with bit i of b
// the measured bit of the i-th upstream cut.  Pauli layout: rows are base-4
// digits (I, X, Y, Z) in the same cut order, columns are x.  A pass changes
// its cuts' row radix to 4 and drops their measured bits from the columns;
// every other index keeps its order.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace tqc {

// tensors with fewer cuts go through the per-entry kernel (a handful of
// terms per entry)
constexpr int kPassMinCuts = 3;

struct TransformSchedule {
  std::vector<TransformPassArgs> passes;  // in / out left null
  uint64_t max_intermediate = 0;          // entries of the largest non-final pass output
};

namespace detail {
struct Axis {
  int kind;   // 0 = measured bit of cut `cut`, 1 = output bits, 2 = row digit of cut `cut`
  int cut;
  uint64_t ext;
};
// axes innermost first with their strides
inline std::vector<Axis> axes_of(const std::vector<int> &rad, const std::vector<int> &bits, int o) {
  std::vector<Axis> ax;
  for (int b : bits) ax.push_back({0, b, 2});
  ax.push_back({1, -1, 1ull << o});
  for (int t = (int)rad.size() - 1; t >= 0; --t) ax.push_back({2, t, (uint64_t)rad[t]});
  return ax;
}
inline uint64_t stride_of(const std::vector<Axis> &ax, int kind, int cut) {
  uint64_t st = 1;
  for (const auto &a : ax) {
    if (a.kind == kind && a.cut == cut) return st;
    st *= a.ext;
  }
  return 0;
}
inline uint64_t total_of(const std::vector<Axis> &ax) {
  uint64_t n = 1;
  for (const auto &a : ax) n *= a.ext;
  return n;
}
}  // namespace detail

inline TransformSchedule transform_schedule(const TensorIn &t) {
  using namespace detail;
  TransformSchedule sc;
  const int c = (int)t.cuts.size(), o = (int)t.outputs.size();
  std::vector<int> rad(c), bits;
  for (int i = 0; i < c; ++i) {
    rad[i] = t.up[i] ? 3 : 4;
    if (t.up[i]) bits.push_back(i);  // measured bits in local cut order, bit 0 first
  }
  // upstream ends first (each pass shrinks the tensor), then downstream
  std::vector<int> seq;
  for (int i = c - 1; i >= 0; --i)
    if (t.up[i]) seq.push_back(i);
  for (int i = 0; i < c; ++i)
    if (!t.up[i]) seq.push_back(i);
  for (size_t p0 = 0; p0 < seq.size(); p0 += 2) {
    const int g = p0 + 1 < seq.size() ? 2 : 1;
    const int pc[2] = {seq[p0], g == 2 ? seq[p0 + 1] : -1};
    const std::vector<Axis> in_ax = axes_of(rad, bits, o);
    std::vector<int> nrad = rad, nbits;
    for (int i = 0; i < g; ++i) nrad[pc[i]] = 4;
    for (int b : bits)
      if (b != pc[0] && b != pc[1]) nbits.push_back(b);
    const std::vector<Axis> out_ax = axes_of(nrad, nbits, o);
    TransformPassArgs a{};
    a.g = g;
    uint64_t fiber = 1;
    for (int i = 0; i < g; ++i) {
      a.up[i] = t.up[pc[i]];
      a.row_in[i] = stride_of(in_ax, 2, pc[i]);
      a.bit_in[i] = a.up[i] ? stride_of(in_ax, 0, pc[i]) : 0;
      a.row_out[i] = stride_of(out_ax, 2, pc[i]);
      fiber *= a.up[i] ? 6 : 4;
    }
    // free segments: maximal runs of the other axes (extent-1 axes skipped)
    uint64_t st = 1;
    bool open = false;
    for (const auto &ax : in_ax) {
      const bool fib = (ax.kind != 1) && (ax.cut == pc[0] || ax.cut == pc[1]);
      if (fib) {
        open = false;
      } else if (ax.ext > 1) {
        if (!open) {
          if (a.nseg == kPassSegs) fail(TQC_ERR_UNSUPPORTED, "transform pass with too many segments");
          a.seg_ext[a.nseg] = 1;
          a.seg_in[a.nseg] = st;
          a.seg_out[a.nseg] = stride_of(out_ax, ax.kind, ax.cut);
          ++a.nseg;
          open = true;
        }
        a.seg_ext[a.nseg - 1] *= ax.ext;
      }
      st *= ax.ext;
    }
    if (a.nseg == 0) {  // every index is a pass index: one free coordinate
      a.seg_ext[0] = 1;
      a.seg_in[0] = a.seg_out[0] = 0;
      a.nseg = 1;
    }
    a.nfree = total_of(in_ax) / fiber;
    a.out_entries = total_of(out_ax);
    sc.passes.push_back(a);
    rad = nrad;
    bits = nbits;
  }
  for (size_t i = 0; i + 1 < sc.passes.size(); ++i)
    sc.max_intermediate = std::max(sc.max_intermediate, sc.passes[i].out_entries);
  return sc;
}

}  // namespace tqc
