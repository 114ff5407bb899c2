// Internal data structures of the tqc library (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tqc.h"

namespace tqc {

// ---------------------------------------------------------------- errors
struct Error {
  tqc_status status;
  std::string msg;
};
[[noreturn]] void fail(tqc_status st, const char *fmt, ...);
void set_last_error(const std::string &msg);

// ------------------------------------------------------------------ labels
// Every index of every tensor is a power of two, so a tensor is a set of
// index bits.  A label names one bit: bit b (0 low, 1 high) of the Pauli
// digit of cut c is 2*c + b; output qubit q is 2*K + q.
inline int cut_label(int c, int b) { return 2 * c + b; }

// -------------------------------------------------------------- network
struct TensorIn {
  std::vector<int> cuts;     // local cut order (first = slowest row digit)
  std::vector<int> outputs;  // qubit of column bit t
  std::vector<int> up;       // per local cut: 1 = upstream (measured) end
  tqc_basis basis = TQC_BASIS_PAULI;
  uint64_t rows = 0, cols = 0;
  std::vector<double> host;
  double maxabs = 0.0;
  int u = 0, d = 0;
  double *dev_raw = nullptr;     // device copy of the input data
  double *dev_pauli = nullptr;   // device Pauli-basis tensor (== dev_raw for PAULI)
  uint64_t pauli_entries() const { return (1ull << (2 * cuts.size())) << outputs.size(); }
};

struct Network {
  int n = 0, m = 0, K = 0;
  std::vector<tqc_cut> cuts;
  std::vector<TensorIn> t;
  int device = -1;
  bool uploaded = false;
  ~Network();
};

// --------------------------------------------------------------------- plan
enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2, BF16X6 = 3, F16X3 = 4 };

struct Node {
  std::vector<int> labels;   // storage layout of the operand form, LSB first
  int kpad_log2 = 0;         // row stride = 2^kpad_log2 elements (>= 2^log2K)
  int log2k = 0;             // k bits at the bottom of the layout
  int producer = -1;         // step producing it (-1: leaf)
  int leaf = -1;             // network tensor for leaves
  bool slice_dep = false;
  int planes = 1;            // bfloat16 split planes
  uint64_t rows = 0;         // 2^(labels above k)
  uint64_t elems() const { return rows << kpad_log2; }
  uint64_t offset = 0;       // byte offset of plane 0 in the workspace
  uint64_t plane_bytes = 0;
};

struct Step {
  int a = -1, b = -1, out = -1;  // node ids
  int lm = 0, ln = 0, lk = 0;    // log2 M, N, K
  int kpad_log2 = 0;             // operand row stride (shared by a and b)
  std::vector<int> m_labels, n_labels, k_labels;
  std::vector<int> posM, posN;   // output bit position of each m / n bit
  bool root = false;
  int tile = 0;
  double flops = 0, bytes = 0;
  int cuts_involved = 0;
};

struct Plan {
  Network *net = nullptr;
  Prec prec = Prec::F32;
  tqc_dtype out_dtype = TQC_F32;
  std::vector<int> fixed_q, fixed_v;
  std::vector<int> sliced;       // sliced cut ids
  std::vector<int> order;        // SSA pairs
  std::vector<Node> nodes;       // 0..m-1 leaves, then one per step
  std::vector<Step> steps;
  std::vector<int> out_labels;   // root output layout (free qubits ascending)
  int out_bits = 0;
  uint64_t num_slices = 1;
  int tile_policy = 0;
  tqc_plan_stats stats{};
  // device state
  int device = -1;
  void *ws = nullptr;
  uint64_t ws_bytes = 0;
  // per tensor: two transform scratch buffers in the workspace (tensors are
  // transformed side by side, so each has its own); bytes of each, 0 = none
  std::vector<uint64_t> tscr_off, tscr_bytes;
  // split-K partial sums of steps whose tiles cannot fill the device
  uint64_t splitk_off = 0, splitk_bytes = 0;
  // float16-split plans: the final step's two operands as float16 planes
  // (hi at h16_off[i], lo one plane later), i = 0 for its A side, 1 for B
  uint64_t h16_off[2] = {0, 0}, h16_plane[2] = {0, 0};
  double *acc64 = nullptr;       // float64 accumulator for sliced runs (when out is f32)
  void *scale_buf = nullptr;     // per-leaf |max| bits, exponents, output scale
  void *stats_buf = nullptr;     // per-tile statistics of the root step + top-k scratch
  uint64_t stats_bytes = 0;
  // caller-owned workspace (tqc_plan_set_workspace): every device buffer
  // above points into it, and scan_buf holds the standalone top-k / total
  // scans of plans without tile statistics; nothing is allocated or freed
  bool ws_external = false;
  void *scan_buf = nullptr;
  uint64_t scan_bytes = 0;
  ~Plan();
};

// planner entry
Plan *build_plan(Network *net, const tqc_plan_options &opt);

// greedy graph growing cut search; returns the number of partitions
int find_cuts(int num_qubits, int num_gates, const int32_t *gate_qubits, int w_max, int s_max, int k_t,
              double q_max, int32_t *labels);

// shapes of the steps a contraction order produces (no layouts)
struct StepShape {
  int lm, ln, lk, kpad, root, slice_dep, tile;
};
std::vector<StepShape> order_shapes(Network *net, Prec prec, const std::vector<int> &sliced,
                                    const std::vector<int> &fixed_q, const std::vector<int> &order);
// candidate orders: the DP / greedy choice, then randomised-greedy samples
std::vector<std::vector<int>> sample_orders(Network *net, Prec prec, tqc_dtype out,
                                            const std::vector<int> &sliced,
                                            const std::vector<int> &fixed_q, int count, uint64_t seed);
int default_tile(int lm, int ln);
int kmin_log2(Prec p);

// plan cost helpers shared with the MLP feature extraction
double prec_peak_flops(Prec p);
int prec_bytes(Prec p);

}  // namespace tqc
