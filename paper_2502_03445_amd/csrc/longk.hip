// Long-k pairwise contractions (Sec. III-B, Eq. (3): a step that closes
// many cuts at once sums over 4^c cut assignments, k >= 512; k >= 256 in
// float64).
//
// Such a step is bound by the matrix cores, and what keeps the MFMA pipes
// idle is memory latency: every workgroup needs a new k slice of both
// operand tiles per MFMA group.  This kernel keeps NS slices in flight:
//   * the operand tiles go from global memory straight into an NS-stage LDS
//     ring (global_load_lds_dwordx4: each lane moves 16 bytes, one
//     instruction fills 1 KiB of LDS), so no registers hold staged data and
//     the ring can be deep;
//   * the slice for stage s + NS is requested while stage s is computed, and
//     one barrier per stage both publishes stage s + 1 and frees the slot of
//     stage s (its fragments are already in registers);
//   * the MFMA fragments of the next k group are read from LDS while the
//     MFMAs of this one run (two register sets); reads, ring loads and MFMAs
//     are issued interleaved, a few MFMAs between consecutive memory
//     instructions, so that a wave never stalls on a full LDS or load queue
//     while it has MFMAs to issue;
//   * rows are stored with their 16-byte chunks XOR-permuted by row, so that
//     fragment reads run without LDS bank conflicts.
// A 128 x 128 output tile per workgroup of four waves (64 x 64 each, as in
// the general kernel); the MFMA sequence per accumulator, the float64 fold of
// every 256-long k chunk (the float32-accumulating forms) and the epilogue
// are those of the general kernel, so both give the same bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_ops.hpp"
#include "kernels.hpp"

namespace tqc {

namespace {

constexpr int kLBM = 128, kLBN = 128;

// Stage depth by form: float64, float32 and the two-plane 16-bit forms move
// 128-byte row slices (16 k of float64 or 32 k of float32 in four 32 KiB
// stages, 64 k of 16-bit values in two 64 KiB stages: every request is one
// whole cache line); the three-plane form moves 64-byte slices (32 k) in
// three 48 KiB stages.
//
// SHORT: the k = 256 variant of float64, float32 and the two-plane forms,
// two workgroups per CU (each hides the other's prologue and epilogue): one
// 256-long chunk, so no float64 fold, and two 32 KiB stages; float64 keeps
// one fragment register set (the other workgroup's waves cover the reads).
template <int P, bool SHORT = false>
struct LongShape {
  using T = PrecTraits<P>;
  static constexpr int NP = T::planes;
  static constexpr int ES = sizeof(typename T::E);
  static constexpr int BK = (P == 0) ? 16 : ((P == 1 || NP == 3 || SHORT) ? 32 : 64);  // k per stage
  static constexpr int KG = T::kgroup;            // k per MFMA group (register set)
  static constexpr int KH = BK / KG;              // MFMA groups per stage
  static constexpr int ROWB = BK * ES;            // bytes of one row's k slice per plane
  static constexpr int CPR = ROWB / 16;           // 16-byte chunks per row slice
  static constexpr int PLANE_B = kLBM * ROWB;     // one operand plane of a stage
  static constexpr int IPP = PLANE_B / 1024;      // 1 KiB load instructions per plane
  static constexpr int STAGE_B = 2 * NP * PLANE_B;
  static constexpr int IPW = STAGE_B / 1024 / 4;  // load instructions per wave per stage
  static constexpr int NS = SHORT ? 2 : ((P <= 1) ? 4 : (NP == 3 ? 3 : 2));
  static constexpr int RING_B = NS * STAGE_B;
  static constexpr int CT_B = kLBM * kLBN * 4;    // staged float tile of the epilogue
  static constexpr int MAIN_B = RING_B > CT_B ? RING_B : CT_B;
  static constexpr int LDS_B = MAIN_B + 64;       // + tile statistics
  static_assert(LDS_B <= (SHORT ? 80 : 160) * 1024, "LDS");
  static_assert(!SHORT || P != 3, "short variant: not the three-plane form");
  static_assert(IPW * 4 * 1024 == STAGE_B && 64 % CPR == 0, "whole instructions");
  static_assert(KH * KG == BK && (KH == 1 || KG * ES == 64), "MFMA groups split a row slice in halves");
};

// XOR permutation of the 16-byte chunks of row r.  A fragment read
// (ds_read_b128) has lane (lr, lg) read row lr of a 16-row block at logical
// chunk lg (+ 4 for the second MFMA group of a 128-byte row; float64 reads
// chunks 2 lg and 2 lg + 1).  The permutations below run these reads
// without LDS bank conflicts on gfx950: the chunk XORed with the row's low
// three bits (float32 and 16-bit planes), with those bits rotated (float64)
// and the pairwise permutation of 64-byte rows (all measured with the LDS
// bank-conflict counter; the identity costs 12 extra cycles per read, most
// other permutations tried 4).
template <int P, int CPR>
__device__ __host__ inline uint32_t chunk_swz(uint32_t r) {
  if constexpr (CPR == 4) return ((r >> 1) ^ (r >> 2)) & 3u;
  else if constexpr (P == 0) return ((r & 3u) << 1) | ((r >> 2) & 1u);
  else return r & 7u;
}

// s_waitcnt immediate (gfx9 layout): vector-memory count v, LDS/scalar count
// l, export count not waited for
constexpr int waitcnt_imm(int v, int l) { return (v & 15) | (7 << 4) | ((l & 15) << 8) | ((v >> 4) << 14); }

// workgroup barrier that does not wait for outstanding vector-memory
// operations (the ring's loads stay in flight across it); the empty asm
// statements keep the compiler from moving memory accesses across it
__device__ inline void ring_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

typedef __attribute__((address_space(3))) void *lds_ptr;

// One workgroup per CU by design (LDS): let the register allocator use the
// whole register file instead of trading latency hiding for occupancy.  The
// short variant runs two per CU and must fit 256 registers per lane.
template <int P, bool SHORT>
__device__ __attribute__((always_inline)) inline void gemm_long_body(const GemmArgs &g, char *smem) {
  using L = LongShape<P, SHORT>;
  constexpr int NP = L::NP, NS = L::NS, CPR = L::CPR, IPW = L::IPW, IPP = L::IPP, KH = L::KH;
  constexpr int FM = 4, FN = 4;

  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t KP = 1ull << g.kpad;
  const uint32_t rowstride = (uint32_t)(KP * L::ES);  // bytes per operand row
  const uint64_t tilesM = M / kLBM, tilesN = N / kLBN;
  uint64_t tm, tn;
  tile_of(blockIdx.x, tilesM, tilesN, g.swz, tm, tn);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  // ---- ring fill: instruction n = j * 4 + wave of a stage writes LDS bytes
  // [n KiB, n + 1 KiB) of the stage: plane region n / IPP = j / (IPP / 4)
  // (A planes, then B planes), rows (n % IPP) * 64 / CPR ..; lane l moves
  // chunk position l % CPR of its row, which holds logical chunk
  // position ^ swz(row)
  static_assert(IPP % 4 == 0, "a plane region is filled by whole rounds of the four waves");
  const char *src[IPW];
  uint32_t soff[IPW];
#pragma unroll
  for (int j = 0; j < IPW; ++j) {
    const int region = j / (IPP / 4), ni = (j % (IPP / 4)) * 4 + wave;
    const uint32_t r = (uint32_t)(ni * (64 / CPR) + lane / CPR);
    const uint32_t c = (uint32_t)(lane % CPR) ^ chunk_swz<P, CPR>(r);
    const bool isA = region < NP;
    const int p = isA ? region : region - NP;
    const void *base = isA ? (p == 0 ? g.a0 : (p == 1 ? g.a1 : g.a2)) : (p == 0 ? g.b0 : (p == 1 ? g.b1 : g.b2));
    const uint64_t row0 = isA ? tm * kLBM : tn * kLBN;
    src[j] = (const char *)base + row0 * rowstride;
    soff[j] = r * rowstride + c * 16u;
  }
  const uint32_t nstages = (uint32_t)(KP / L::BK);
  auto issue_one = [&](uint32_t s, int j) {
    char *slot = smem + (s % NS) * L::STAGE_B;
    __builtin_amdgcn_global_load_lds((const void *)(src[j] + s * (uint32_t)L::ROWB + soff[j]),
                                     (lds_ptr)(slot + (j * 4 + wave) * 1024), 16, 0, 0);
  };
  auto issue = [&](uint32_t s) {
    char *slot = smem + (s % NS) * L::STAGE_B;
    const uint32_t kb = s * (uint32_t)L::ROWB;
#pragma unroll
    for (int j = 0; j < IPW; ++j)
      __builtin_amdgcn_global_load_lds((const void *)(src[j] + kb + soff[j]),
                                       (lds_ptr)(slot + (j * 4 + wave) * 1024), 16, 0, 0);
  };

  // ---- fragment reads: lane (lr, lg) of block i reads row wm*64 + i*16 + lr,
  // logical chunk 4h + lg for MFMA group h of the stage
  constexpr int FH0 = (P == 0) ? 2 : 1;  // 16-byte chunks per fragment of one lane
  uint32_t aoff[FM], boff[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const uint32_t r = (uint32_t)(wm * 64 + i * 16 + lr);
    aoff[i] = r * L::ROWB + (((uint32_t)(lg * FH0) ^ chunk_swz<P, CPR>(r)) * 16u);
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const uint32_t r = (uint32_t)(wn * 64 + j * 16 + lr);
    boff[j] = NP * L::PLANE_B + r * L::ROWB + (((uint32_t)(lg * FH0) ^ chunk_swz<P, CPR>(r)) * 16u);
  }

  using Acc = typename PrecTraits<P>::Acc;  // float64 accumulates in place, no fold
  Acc acc[FM][FN];
  doublex4 acc2[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      acc2[i][j] = doublex4{0, 0, 0, 0};
    }

  // two register sets, one MFMA group (16 k of float64 or float32, 32 k of
  // 16-bit values) each; group x = stage x / KH, part x % KH.  A float64
  // fragment (four k of one row, 32 bytes) is two 16-byte reads: logical
  // chunks 2 lg and 2 lg + 1, i.e. positions p and p ^ 1.
  using Frag = typename std::conditional<P == 1, floatx4, typename std::conditional<P == 0, double2v, bf16x8>::type>::type;
  constexpr int FH = (P == 0) ? 2 : 1;  // 16-byte reads per fragment
  constexpr bool ONESET = P == 0 && SHORT;
  constexpr int NSET = ONESET ? 1 : 2;
  Frag fa[NSET][NP][FM][FH], fb[NSET][NP][FN][FH];
  auto read_one = [&](auto SET, const char *st, uint32_t hx, int k) {
    constexpr int q = decltype(SET)::value;
    const int h = k % FH, f = k / FH, p = f / 8, w = f % 8;
    const uint32_t hb = (uint32_t)h * 16u;
    if (w < 4) fa[q][p][w][h] = *(const Frag *)(st + p * L::PLANE_B + ((aoff[w] ^ hx) ^ hb));
    else fb[q][p][w - 4][h] = *(const Frag *)(st + p * L::PLANE_B + ((boff[w - 4] ^ hx) ^ hb));
  };
  auto read_frags = [&](auto SET, uint32_t x) {
    const char *st = smem + ((x / KH) % NS) * L::STAGE_B;
    const uint32_t hx = (x % KH) * 64u;
#pragma unroll
    for (int k = 0; k < NP * 8 * FH; ++k) read_one(SET, st, hx, k);
  };
  // MFMA m of a group, in the order of the general kernel per accumulator:
  // float32 by k step t, then blocks; the split forms by product, then blocks
  constexpr int NREAD = NP * (FM + FN) * FH;             // 16-byte reads per group
  constexpr int NMF = (P <= 1) ? 64 : ((NP == 3) ? 96 : 48);  // MFMAs per group
  constexpr int MPS = NMF / NREAD;                       // MFMAs per slot
  static_assert(MPS * NREAD == NMF && IPW <= NREAD, "slots");
  auto mfma_one = [&](auto SET, int m) {
    constexpr int q = decltype(SET)::value;
    const int i = (m / 4) % 4, j = m % 4;
    if constexpr (P == 0) {
      const int t = m / 16;
      acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q][0][i][t / 2][t % 2], fb[q][0][j][t / 2][t % 2], acc[i][j], 0,
                                                      0, 0);
    } else if constexpr (P == 1) {
      const int t = m / 16;
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[q][0][i][0][t], fb[q][0][j][0][t], acc[i][j], 0, 0, 0);
    } else {
      constexpr int pa3[6] = {2, 1, 0, 1, 0, 0}, pb3[6] = {0, 1, 2, 0, 1, 0};
      constexpr int pa2[3] = {1, 0, 0}, pb2[3] = {0, 1, 0};
      const int pr = m / 16;
      const int x = (NP == 3) ? pa3[pr] : pa2[pr];
      const int y = (NP == 3) ? pb3[pr] : pb2[pr];
      acc[i][j] = mfma_split<P>(fa[q][x][i][0], fb[q][y][j][0], acc[i][j]);
    }
  };
  auto fold = [&]() {
    if constexpr (P == 0 || SHORT) return;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc2[i][j][r] += (double)acc[i][j][r];
        acc[i][j] = Acc{0, 0, 0, 0};
      }
  };

  // prologue: stages 0 .. NS - 1 requested, group 0 in registers
#pragma unroll
  for (int s = 0; s < NS; ++s) issue((uint32_t)s);
  __builtin_amdgcn_s_waitcnt(waitcnt_imm((NS - 1) * IPW, 15));
  ring_barrier();
  read_frags(std::integral_constant<int, 0>{}, 0);

  // group x = c * GPC + u of fold chunk c (256 k): read group x + 1 while
  // the MFMAs of group x run.  When x + 1 starts stage s + 1: wait for stage
  // s + 1 (and for this wave's reads of stage s), barrier, request stage
  // s + NS into the slot of stage s.  After the last group the read of
  // "group x + 1" touches a stale slot whose values are never used.
  constexpr int GPC = 256 / L::KG;  // MFMA groups per float64 fold
  static_assert(GPC % 2 == 0 && GPC % KH == 0, "chunks hold whole stages and register-set pairs");
  const uint32_t nchunks = (uint32_t)(KP / 256);
  for (uint32_t c = 0; c < nchunks; ++c) {
#pragma unroll
    for (int u = 0; u < GPC; ++u) {
      const uint32_t x = c * GPC + (uint32_t)u;
      // the reads of group x have had a whole MFMA group to land: wait for
      // them before the reads of group x + 1 are issued (the LDS counter
      // cannot express "all but the last 16")
      __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
      bool dma_here = false;
      if ((u + 1) % KH == 0) {
        const uint32_t s = x / KH;
        if (s + NS - 1 < nstages) __builtin_amdgcn_s_waitcnt(waitcnt_imm((NS - 2) * IPW, 0));
        else __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));
        ring_barrier();
        dma_here = s + NS < nstages;
      }
      // slots: read k of group x + 1, ring load k (at a stage boundary),
      // then MPS MFMAs of group x; each slot closed by a scheduling fence
      const uint32_t xn = x + 1;
      const char *stn = smem + ((xn / KH) % NS) * L::STAGE_B;
      const uint32_t hx = (xn % KH) * 64u;
      const uint32_t sN = x / KH + NS;
      auto body = [&](auto SET) {
        constexpr int q = decltype(SET)::value;
#pragma unroll
        for (int k = 0; k < NREAD; ++k) {
          read_one(std::integral_constant<int, 1 - q>{}, stn, hx, k);
          if (k < IPW && dma_here) issue_one(sN, k < IPW ? k : 0);
#pragma unroll
          for (int m = k * MPS; m < (k + 1) * MPS; ++m) mfma_one(SET, m);
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      // one register set: this group's MFMAs (with the ring loads between
      // them), then the reads of the next group into the same registers
      auto body1 = [&]() {
        constexpr auto S0 = std::integral_constant<int, 0>{};
#pragma unroll
        for (int k = 0; k < NREAD; ++k) {
          if (k < IPW && dma_here) issue_one(sN, k < IPW ? k : 0);
#pragma unroll
          for (int m = k * MPS; m < (k + 1) * MPS; ++m) mfma_one(S0, m);
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < NREAD; ++k) read_one(S0, stn, hx, k);
        __builtin_amdgcn_sched_barrier(0);
      };
      if constexpr (ONESET) body1();
      else if (u & 1) body(std::integral_constant<int, 1>{});
      else body(std::integral_constant<int, 0>{});
    }
    fold();
  }

  const bool staged = P != 0 && g.staged && g.out_kind != OUT_F64 && g.out_kind != OUT_F64_ACC;
  auto result = [&](int i, int j, int r) -> double {
    if constexpr (P == 0 || SHORT) return acc[i][j][r];
    else return acc2[i][j][r];
  };
  gemm_epilogue<P, kLBM, kLBN>(g, smem, L::MAIN_B, tm, tn, 0, staged, result);
}

template <int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) gemm_long_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(1024))) char smem[LongShape<P>::LDS_B];
  gemm_long_body<P, false>(g, smem);
}

template <int P>
__global__ void __launch_bounds__(256, 2) __attribute__((amdgpu_waves_per_eu(2, 2))) gemm_short_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(1024))) char smem[LongShape<P, true>::LDS_B];
  gemm_long_body<P, true>(g, smem);
}

template <int P, bool SHORT>
hipError_t launch_long_t(GemmArgs g, hipStream_t s) {
  using L = LongShape<P, SHORT>;
  const uint64_t tiles = (1ull << g.lm) / kLBM * ((1ull << g.ln) / kLBN);
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  // the prologue requests NS stages, and k runs in whole 256-long chunks
  // (exactly one for the short variant)
  if (g.kpad < 8 || ((1ull << g.kpad) / L::BK) < (uint64_t)L::NS) return hipErrorInvalidValue;
  if (SHORT && g.kpad != 8) return hipErrorInvalidValue;
  prepare_gemm_args(g, P, kLBM, kLBN);
  g.ksplit = 0;
  if constexpr (SHORT)
    hipLaunchKernelGGL(gemm_short_kernel<P>, dim3((unsigned)tiles), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(gemm_long_kernel<P>, dim3((unsigned)tiles), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

bool gemm_long_eligible(int prec, const GemmArgs &g, uint64_t min_tiles) {
  if (prec < 0 || prec > 4) return false;
  // k >= 256 on whole 128 x 128 tiles.  At k = 256 the one-workgroup-per-CU
  // kernel loses to the general kernel, whose two workgroups per CU hide
  // their prologue and epilogue behind each other's MFMAs (measured), except
  // in float64, where the general kernel runs one per CU as well; the other
  // forms take the short variant there (two per CU), bf16x6 (too many
  // registers for it) keeps the general kernel.
  if (g.kpad < (prec == 3 ? 9 : 8) || g.lm < 7 || g.ln < 7) return false;
  // 32-bit row offsets within a tile: 127 rows x 2^22 k x 8 bytes < 2^32
  if ((uint64_t)1 << g.kpad > (1ull << 22)) return false;
  const uint64_t tiles = (1ull << (g.lm - 7)) << (g.ln - 7);
  return tiles >= min_tiles;
}

hipError_t launch_gemm_long(int prec, const GemmArgs &g, hipStream_t s) {
  const bool sh = g.kpad == 8;
  switch (prec) {
    case 0: return sh ? launch_long_t<0, true>(g, s) : launch_long_t<0, false>(g, s);
    case 1: return sh ? launch_long_t<1, true>(g, s) : launch_long_t<1, false>(g, s);
    case 2: return sh ? launch_long_t<2, true>(g, s) : launch_long_t<2, false>(g, s);
    case 3: return launch_long_t<3, false>(g, s);
    case 4: return sh ? launch_long_t<4, true>(g, s) : launch_long_t<4, false>(g, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tqc
