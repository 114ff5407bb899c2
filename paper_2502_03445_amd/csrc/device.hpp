// Device-side helpers and kernel argument structs shared by the kernels and
// the executor.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tqc {

constexpr int kMaxBits = 48;   // index bits per tensor
constexpr int kMaxCutsT = 16;  // cuts per raw tensor in the transform kernel

// ------------------------------------------------------------- bfloat16
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// ----------------------------------------------------------- transform
// Direct form of the Pauli-basis transform for one raw tensor: every output
// element T[sigma][x] is a signed sum over the measured cut bits of the
// upstream cuts and the two or three preparations that build each Pauli on
// the downstream cuts.
struct TransformArgs {
  const double *raw;
  double *out;
  int c, o, u;
  int up[kMaxCutsT];        // 1 if upstream end
  int bbit[kMaxCutsT];      // upstream: index of its measured bit in b
  uint64_t w[kMaxCutsT];    // mixed-radix weight of the cut's raw row digit
  // optional (amax non-null): the largest |value| written among the entries
  // whose index bits under amask equal abase (the fixed output qubits), as
  // float64 bits, atomically maxed into *amax
  unsigned long long *amax;
  uint64_t amask, abase;
};

// One pass of the separable Pauli transform: one or two cuts of a tensor
// change from their measured / prepared variants to Pauli digits, every
// other index is a free coordinate.  A free coordinate splits, innermost
// first, into segments of extent seg_ext; each segment's digit moves the
// source and destination by seg_in / seg_out elements.  For pass cut i the
// source holds its variants at multiples of row_in[i] (row digit: basis or
// preparation) and bit_in[i] (the measured bit of an upstream end); the
// destination holds its Pauli digit at multiples of row_out[i].
constexpr int kPassSegs = 5;
constexpr int kPassBatch = 8;   // passes per launch
constexpr int kPackBatch = 8;   // leaves per pack / abs-max launch
struct TransformPassArgs {
  const double *in;
  double *out;
  uint64_t nfree;
  int nseg;
  int g;                      // cuts in the pass (1 or 2)
  int up[2];                  // 1 = upstream end
  uint64_t seg_ext[kPassSegs], seg_in[kPassSegs], seg_out[kPassSegs];
  uint64_t row_in[2], bit_in[2], row_out[2];
  uint64_t out_entries;       // destination size (for host-side checks)
  unsigned long long *amax;   // optional abs-max of the written entries, as
  uint64_t amask, abase;      // in TransformArgs (a tensor's last pass only)
};

// ---------------------------------------------------------------- pack
// Gather one leaf operand from its float64 Pauli tensor: slice / fixed-qubit
// selection via a base offset, arbitrary bit permutation, cast or split.
struct PackArgs {
  const double *src;
  void *dst0, *dst1, *dst2;  // planes
  uint64_t base;             // source offset of the fixed bits
  int nbits;                 // destination index bits (k bits first)
  int lk, kpad;              // k bits and padded row stride (log2)
  int inpos[kMaxBits];       // source bit position of destination bit i
  int prec;                  // 0 f64, 1 f32, 2 bf16x2 split, 3 bf16x3 split
  double scale;              // exact power of two
  const int *dexp;           // optional device exponent e: values scaled by 2^e
  const unsigned long long *dmax;  // optional device abs-max bits (instead of
                                   // dexp): e = -floor(log2 max), 0 if max = 0
  // optional tiling (tkb > 0): a workgroup moves the entries whose
  // destination bits 0..tkb-1 and source bits 0..tsb-1 vary through LDS;
  // source bit t < tsb is destination bit dpos[t]; the workgroup's tile
  // index fills the destination index bits in tmask (the others)
  int tkb, tsb;
  int8_t dpos[8];
  uint64_t tmask;
};

// Largest |value| of a leaf operand over every slice (the gathered bits plus
// the sliced-cut bits), as the bit pattern of a non-negative double.
struct AbsMaxArgs {
  const double *src;
  uint64_t base;             // fixed-qubit bits
  int nbits;
  int inpos[kMaxBits];
  unsigned long long *out;
};

// ---------------------------------------------------------------- GEMM
enum OutKind : int {
  OUT_F64 = 0,
  OUT_F32 = 1,
  OUT_SPLIT2 = 2,  // bfloat16 hi/lo planes
  OUT_SPLIT3 = 3,  // bfloat16 hi/mid/lo planes
  OUT_F64_ACC = 4, // float64 +=
};

struct GemmArgs {
  const void *a0, *a1, *a2;  // operand A planes, [M][2^kpad]
  const void *b0, *b1, *b2;  // operand B planes, [N][2^kpad]
  void *c0, *c1, *c2;        // output planes
  int lm, ln, lk, kpad;
  int out_kind;
  double scale;
  const double *dscale;      // optional device scale (overrides scale)
  uint8_t posM[kMaxBits];
  uint8_t posN[kMaxBits];
  // filled by the launcher for the chosen tile (staged epilogue):
  int staged;                // 1: full tiles, stage C through LDS
  int vec4;                  // compact bits 0,1 are output bits 0,1
  int ncompact;              // log2(BM) + log2(BN)
  uint8_t rankM[16], rankN[16];  // compact bit of tile-local row / col bit i
  uint8_t lpos[32];          // output bit of compact bit b
  int swz;                   // XCD-aware tile order
  // optional per-tile statistics of the stored values (root step only):
  // largest order-preserving key and float64 sum, at tile tm * tilesN + tn
  unsigned long long *tkey;
  double *tsum;
  // split-K: with ksplit > 0 each workgroup sums one of 2^ksplit equal k
  // ranges of one tile and writes float64 partial results to
  // partial[(split * M + m) * N + n]; a reduction adds the splits in order
  // and applies the epilogue.  partial_bytes bounds the split count.
  double *partial;
  uint64_t partial_bytes;
  int ksplit;
};

}  // namespace tqc
