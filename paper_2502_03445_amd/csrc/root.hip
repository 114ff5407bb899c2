// Persistent final contraction for short K (Sec. III-B, the last pairwise
// step writes the 2^n output).
//
// The last step of a reconstruction is a GEMM with a huge M x N (the output)
// and a short K (4^c for the c cuts it closes), so its cost is storing the
// output plus the MFMA work, and both must run at once.  One workgroup of
// eight waves per CU loops over 128 x 128 output tiles; the waves split the
// work by role, one of each role per SIMD:
//   * four MFMA waves load operand fragments from global memory straight into
//     the MFMA register layout (no LDS), a fragment group ahead of their use,
//     and write the accumulators of tile i to staged tile buffer i & 1 in LDS;
//   * four store waves convert staged tile i - 1, store it to HBM in output
//     order (float4 runs) and reduce its per-tile statistics;
//   * one barrier per tile hands the buffers over.
// So the MFMA pipe and the store stream run at the same time on every SIMD.
// Tiles are split into eight contiguous ranges, one per XCD (workgroup ids
// go round-robin over the XCDs); the workgroups of one XCD walk their range
// in groups of eight tile rows, column by column, so the tiles in flight on
// an XCD share A and B blocks in its L2.  The arithmetic per accumulator is the same sequence as in
// the general GEMM kernel, so results agree bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dev_ops.hpp"
#include "kernels.hpp"

namespace tqc {

namespace {

constexpr int kRT = 128;                   // tile edge
constexpr int kCtBytes = kRT * kRT * 4;    // one staged float tile
constexpr int kStatOff = 2 * kCtBytes;     // sums [2][4] doubles, then keys [2][4] (16-byte rows)
constexpr int kRootLds = kStatOff + 256;

// 16-byte chunk swizzle of the staged tile: higher compact bits are folded
// into bits 2..4 so that the scattered single-float writes of the MFMA
// layout spread over the LDS banks; float4 reads at multiples of 4 stay
// contiguous.
__device__ inline uint32_t ct_swz(uint32_t c) {
  return c ^ ((((c >> 5) ^ (c >> 8) ^ (c >> 11)) & 7u) << 2);
}

template <int P>
struct RootTraits;
template <>
struct RootTraits<1> {
  static constexpr int KG = 16;  // k per fragment group (4 MFMAs of k = 4)
  static constexpr int NP = 1;
  static constexpr int ES = 4;
  using Frag = floatx4;
};
template <>
struct RootTraits<2> {
  static constexpr int KG = 32;
  static constexpr int NP = 2;
  static constexpr int ES = 2;
  using Frag = bf16x8;
};
template <>
struct RootTraits<3> {
  static constexpr int KG = 32;
  static constexpr int NP = 3;
  static constexpr int ES = 2;
  using Frag = bf16x8;
};
template <>
struct RootTraits<4> {  // two float16 planes: the bf16x3 schedule on float16 MFMA
  static constexpr int KG = 32;
  static constexpr int NP = 2;
  static constexpr int ES = 2;
  using Frag = bf16x8;  // 16-bit lanes; mfma_split<4> reads them as float16
};

// Workgroup barrier ordering LDS only.  __syncthreads() also waits for every
// outstanding global store of the wave, which would drain the output store
// stream at each tile; nothing here reads global memory written by another
// wave of the kernel.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// OR of v over the 64 lanes of the wave (the result is wave-uniform)
__device__ inline uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

// MULTI: one launch for the final steps of many reconstructions that share
// the form and K; blockIdx.y selects the job, whose arguments and tile
// counts come from a device table, and blockIdx.x plays the role of the
// workgroup id of a single-job launch of gridDim.x workgroups.
template <int P, int KP, bool STATS, bool MULTI>
__global__ void __launch_bounds__(512) root_gemm_kernel(GemmArgs g_in, uint32_t ntiles_in, int lgtm_in, int lgtn_in,
                                                        const RootJob *jobs) {
  const GemmArgs &g = MULTI ? jobs[blockIdx.y].g : g_in;
  const uint32_t ntiles = MULTI ? jobs[blockIdx.y].ntiles : ntiles_in;
  const int lgtm = MULTI ? jobs[blockIdx.y].lgtm : lgtm_in;
  const int lgtn = MULTI ? jobs[blockIdx.y].lgtn : lgtn_in;
  using RT = RootTraits<P>;
  using Frag = typename RT::Frag;
  constexpr int KG = RT::KG, NP = RT::NP, ES = RT::ES;
  constexpr int NKG = KP / KG;
  constexpr int RMAX = (NP == 3) ? 1 : 2;     // fragment groups in flight (256 VGPRs per lane)
  constexpr int R = NKG < RMAX ? NKG : RMAX;
  static_assert(NKG >= 1 && NKG % R == 0, "k groups");
  constexpr int FM = 4, FN = 4;  // 16 x 16 blocks per MFMA wave (64 x 64 sub-tile)

  __shared__ __attribute__((aligned(16))) char smem[kRootLds];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform role

  // this workgroup's tiles: XCD range [r0, r1), every nslots-th from slot
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t xcd = b & 7u, slot = b >> 3;
  const uint32_t nslots = (G - xcd + 7u) >> 3;
  const uint32_t per = (ntiles + 7u) >> 3;
  const uint32_t r0 = xcd * per;
  const uint32_t r1 = r0 + per < ntiles ? r0 + per : ntiles;
  const uint32_t mine = r1 > r0 + slot ? (r1 - r0 - slot + nslots - 1) / nslots : 0;
  if (mine == 0) return;  // whole workgroup, before any barrier
  // walk order: groups of GM tile rows, column by column inside a group, so
  // the tiles in flight on an XCD share GM A row-blocks (kept in its L2) and
  // each B column-block is fetched once per group
  const uint32_t tnmask = (1u << lgtn) - 1;
  const int lgm = lgtm < 3 ? lgtm : 3;
  auto tile_at = [&](uint32_t i) {
    const uint32_t idx = r0 + slot + i * nslots;
    const uint32_t grp = idx >> (lgm + lgtn), r = idx & ((1u << (lgm + lgtn)) - 1);
    const uint32_t tm = (grp << lgm) | (r & ((1u << lgm) - 1)), tn = r >> lgm;
    return (tm << lgtn) | tn;
  };

  if (wave < 4) {
    // ---------------- MFMA waves: tile i into staged buffer i & 1
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lg = lane >> 4;
    const char *Ap[3] = {(const char *)g.a0, (const char *)g.a1, (const char *)g.a2};
    const char *Bp[3] = {(const char *)g.b0, (const char *)g.b1, (const char *)g.b2};
    // A row-blocks repeat along a walk (the same tile row for many tiles):
    // when they fit, all k groups of A stay in registers and only B streams
    constexpr bool HOLD_A = NKG * NP * FM * 4 <= (NP == 3 ? 96 : 64);
    constexpr int NA = HOLD_A ? NKG : R;
    Frag fa[NA][NP][FM], fb[R][NP][FN];
    floatx4 acc[FM][FN];
    auto a_off = [&](uint32_t tile) {
      return ((uint64_t)(tile >> lgtn) * kRT + wm * 64 + lr) * (uint64_t)(KP * ES) + 16 * lg;
    };
    auto b_off = [&](uint32_t tile) {
      return ((uint64_t)(tile & tnmask) * kRT + wn * 64 + lr) * (uint64_t)(KP * ES) + 16 * lg;
    };
    auto load_a = [&](uint64_t ao, int kg, int q) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
          fa[q][p][i] = *(const Frag *)(Ap[p] + ao + (uint64_t)(i * 16 * KP + kg * KG) * ES);
    };
    auto load_b = [&](uint64_t bo, int kg, int q) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fb[q][p][j] = *(const Frag *)(Bp[p] + bo + (uint64_t)(j * 16 * KP + kg * KG) * ES);
    };
    auto mfma_group = [&](int qa, int q) {
      if constexpr (P == 1) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[qa][0][i][t], fb[q][0][j][t], acc[i][j], 0, 0, 0);
      } else {
        // products smallest first, the same order per accumulator as the
        // general kernel; all 16 accumulators between dependent MFMAs
        constexpr int NPR = (NP == 3) ? 6 : 3;
        constexpr int pa3[6] = {2, 1, 0, 1, 0, 0}, pb3[6] = {0, 1, 2, 0, 1, 0};
        constexpr int pa2[3] = {1, 0, 0}, pb2[3] = {0, 1, 0};
#pragma unroll
        for (int pr = 0; pr < NPR; ++pr) {
          const int x = (NP == 3) ? pa3[pr] : pa2[pr];
          const int y = (NP == 3) ? pb3[pr] : pb2[pr];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = mfma_split<P>(fa[qa][x][i], fb[q][y][j], acc[i][j]);
        }
      }
    };
    // tile-local row / column -> swizzled compact (output-ordered) index
    // (the swizzle is XOR-linear and row / column bits are disjoint, so the
    // swizzled index is the XOR of a row part and a column part)
    // Deposits of disjoint bits add up, so the index splits further into a
    // per-lane part (lane row / column bits) and wave-uniform parts per
    // (i, r) and j, kept in scalar registers.
    const uint32_t ctlane = 4 * ct_swz((uint32_t)deposit_c<7>(wm * 64 + 4 * lg, g.rankM, 7)) ^
                            4 * ct_swz((uint32_t)deposit_c<7>(wn * 64 + lr, g.rankN, 7));
    auto trow = [&](int i, int r) { return 4 * ct_swz((uint32_t)deposit_c<7>(i * 16 + r, g.rankM, 7)); };
    auto tcol = [&](int j) { return 4 * ct_swz((uint32_t)deposit_c<7>(j * 16, g.rankN, 7)); };
    {
      const uint64_t bo = b_off(tile_at(0));
#pragma unroll
      for (int q = 0; q < R; ++q) {
        if constexpr (!HOLD_A) load_a(a_off(tile_at(0)), q, q);
        load_b(bo, q, q);
      }
    }
    // one tile: MFMAs of `cur` while the next fragment groups (the last ones
    // for tile `next`) load, then its accumulators to staged buffer `it & 1`
    auto tile_step = [&](uint32_t it) {
      const uint32_t cur = tile_at(it), next = tile_at(it + 1 < mine ? it + 1 : it);
      const uint64_t ca = a_off(cur), cb = b_off(cur), na = a_off(next), nb = b_off(next);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
#pragma unroll
      for (int kg = 0; kg < NKG; ++kg) {
        const int q = kg % R;
        mfma_group(HOLD_A ? kg : q, q);
        if (kg + R < NKG) {
          if constexpr (!HOLD_A) load_a(ca, kg + R, q);
          load_b(cb, kg + R, q);
        } else {
          if constexpr (!HOLD_A) load_a(na, kg + R - NKG, q);
          load_b(nb, kg + R - NKG, q);
        }
        // keep the prefetch here: the scheduler would otherwise sink the
        // loads next to their use and expose their latency
        __builtin_amdgcn_sched_barrier(0);
      }
      char *ct = smem + (it & 1) * kCtBytes;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            *(float *)(ct + (ctlane ^ trow(i, r) ^ tcol(j))) = acc[i][j][r];
      lds_barrier();
    };
    if constexpr (HOLD_A && P != 1) {
      // Column-slice pipeline: unit u = (tile u / NSL, column slice u % NSL).
      // The MFMAs of unit u run while the accumulators of unit u - 1 go to
      // the staged tile, so the staging writes overlap the math; the barrier
      // that hands a tile to the store waves follows the write of its last
      // slice.  Narrower slices for bf16x6 keep its registers in budget.
      constexpr int NSL = (NP == 3) ? 4 : 2;
      constexpr int FH = FN / NSL;
      // B fragment groups in flight: the ring runs across slices and tiles
      constexpr int RSMAX = 2;
      constexpr int RS = NSL * NKG < RSMAX ? NSL * NKG : RSMAX;
      static_assert((NSL * NKG) % RS == 0, "ring aligned with tiles");
      Frag fbh[RS][NP][FH];
      floatx4 ah[2][FM][FH];
      const uint32_t nunits = NSL * mine;
      // B address = wave-uniform part (tile column block and slice: scalar
      // registers) + a 32-bit per-lane part fixed for the whole kernel
      const uint32_t blane = (uint32_t)(wn * 64 + lr) * (uint32_t)(KP * ES) + 16u * lg;
      auto bh_off = [&](uint32_t u) {
        const uint32_t tile = tile_at(u / NSL);
        return ((uint64_t)(tile & tnmask) * kRT + (u % NSL) * (64 / NSL)) * (uint64_t)(KP * ES);
      };
      auto load_bh = [&](uint64_t bo, int kg, int q) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const char *bp = Bp[p] + bo;
#pragma unroll
          for (int j = 0; j < FH; ++j)
            fbh[q][p][j] = *(const Frag *)(bp + blane + (uint32_t)((j * 16 * KP + kg * KG) * ES));
        }
      };
      auto mfma_half = [&](int sa, int kg, int q) {
        if constexpr (P == 1) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
              for (int j = 0; j < FH; ++j)
                ah[sa][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[kg][0][i][t], fbh[q][0][j][t], ah[sa][i][j], 0, 0, 0);
        } else {
          constexpr int NPR = (NP == 3) ? 6 : 3;
          constexpr int pa3[6] = {2, 1, 0, 1, 0, 0}, pb3[6] = {0, 1, 2, 0, 1, 0};
          constexpr int pa2[3] = {1, 0, 0}, pb2[3] = {0, 1, 0};
#pragma unroll
          for (int pr = 0; pr < NPR; ++pr) {
            const int x = (NP == 3) ? pa3[pr] : pa2[pr];
            const int y = (NP == 3) ? pb3[pr] : pb2[pr];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
              for (int j = 0; j < FH; ++j)
                ah[sa][i][j] = mfma_split<P>(fa[kg][x][i], fbh[q][y][j], ah[sa][i][j]);
          }
        }
      };
      auto write_half = [&](uint32_t u, int sa) {
        char *ct = smem + ((u / NSL) & 1) * kCtBytes;
        const int h = (int)(u % NSL);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < FH; ++j)
              *(float *)(ct + (ctlane ^ trow(i, r) ^ tcol(h * FH + j))) = ah[sa][i][j][r];
      };
      // compute unit u into ah[u & 1] (prefetching the next unit's B groups);
      // with PREV, also stage unit u - 1 from ah[(u - 1) & 1]
      // unit u is slice SI of its tile; its k groups are ring slots
      // (SI * NKG + kg) % RS, refilled RS groups ahead
      auto unit_step = [&](auto PREV, auto SA, auto SI, uint32_t u) {
        constexpr bool WR = decltype(PREV)::value;
        constexpr int sa = decltype(SA)::value;  // = u & 1, compile-time register set
        constexpr int si = decltype(SI)::value;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FH; ++j) ah[sa][i][j] = floatx4{0, 0, 0, 0};
#pragma unroll
        for (int kg = 0; kg < NKG; ++kg) {
          const int gidx = si * NKG + kg;
          const int q = gidx % RS;
          mfma_half(sa, kg, q);
          {
            const int G = gidx + RS;
            const uint32_t ut = u - si + G / NKG;
            load_bh(bh_off(ut < nunits ? ut : nunits - 1), G % NKG, q);
          }
          if constexpr (WR) {
            if (kg == 0) write_half(u - 1, sa ^ 1);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (WR) {
          if (u % NSL == 0) lds_barrier();  // unit u - 1 completed tile (u - 1) / NSL
        }
      };
      using T1h = std::true_type;
      using F0h = std::false_type;
      using S0 = std::integral_constant<int, 0>;
      using S1 = std::integral_constant<int, 1>;
      {
#pragma unroll
        for (int q = 0; q < RS; ++q) load_bh(bh_off((uint32_t)(q / NKG) < nunits ? q / NKG : nunits - 1), q % NKG, q);
      }
      // runs of units in one tile row: A loaded once per run, outside the
      // inner loop, so the inner loop has no conditional loads
      uint32_t it = 0;
      while (it < mine) {
        const uint32_t tm_run = tile_at(it) >> lgtn;
        const uint64_t ao = a_off(tile_at(it));
#pragma unroll
        for (int q = 0; q < NA; ++q) load_a(ao, q, q);
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        auto tile_units = [&](auto FIRST, uint32_t t) {
          if constexpr (decltype(FIRST)::value) unit_step(F0h{}, S0{}, I0{}, NSL * t);
          else unit_step(T1h{}, S0{}, I0{}, NSL * t);
          unit_step(T1h{}, S1{}, I1{}, NSL * t + 1);
          if constexpr (NSL == 4) {
            unit_step(T1h{}, S0{}, I2{}, NSL * t + 2);
            unit_step(T1h{}, S1{}, I3{}, NSL * t + 3);
          }
        };
        if (it == 0) {
          tile_units(T1h{}, 0);
          ++it;
        }
        while (it < mine && (tile_at(it) >> lgtn) == tm_run) {
          tile_units(F0h{}, it);
          ++it;
        }
      }
      write_half(nunits - 1, 1);
      lds_barrier();
    } else if constexpr (HOLD_A) {
      // (float32 operands: the MFMA pipe is the bound and the whole-tile
      // order measured faster than the half-tile pipeline)
      // runs of consecutive tiles in one tile row: A loaded once per run,
      // outside the inner loop, so the inner loop has no conditional loads
      uint32_t it = 0;
      while (it < mine) {
        const uint32_t tm_run = tile_at(it) >> lgtn;
        const uint64_t ao = a_off(tile_at(it));
#pragma unroll
        for (int q = 0; q < NA; ++q) load_a(ao, q, q);
        do {
          tile_step(it);
          ++it;
        } while (it < mine && (tile_at(it) >> lgtn) == tm_run);
      }
    } else {
      for (uint32_t it = 0; it < mine; ++it) tile_step(it);
    }
    lds_barrier();
  } else {
    // ---------------- store waves: staged tile i - 1 to the output
    const int et = tid - 256, ew = wave - 4;
    // the output scale is a power of two (2^-K times the operand exponents):
    // ldexp rounds once, like the float64 product rounded to float32
    const int sexp = ilogb(g.dscale ? *g.dscale : g.scale);
    // compact index x = c * 1024 + et * 4 + e lands at base + lo + hi(c) + e
    const uint64_t lo = deposit_c<10>((uint64_t)et * 4, g.lpos, 10);
    const uint32_t xlo = 4 * ct_swz((uint32_t)et * 4u);
    // output offset of a tile's first entry: lane l deposits bit 7 + l of
    // the tile row and of the tile column, then the wave ORs them together
    const int pm = 7 + lane < g.lm ? g.posM[7 + lane] : 0;
    const int pn = 7 + lane < g.ln ? g.posN[7 + lane] : 0;
    const bool hm = 7 + lane < g.lm, hn = 7 + lane < g.ln;
    auto tile_base = [&](uint32_t tile) {
      const uint32_t tm = tile >> lgtn, tn = tile & tnmask;
      uint64_t v = 0;
      if (hm && lane < 32 && ((tm >> lane) & 1u)) v |= 1ull << pm;
      if (hn && lane < 32 && ((tn >> lane) & 1u)) v |= 1ull << pn;
      return wave_or(v);
    };
    auto combine = [&](uint32_t tile, int par) {
      const double *rs = (const double *)(smem + kStatOff + par * 64);
      const uint32_t *rk = (const uint32_t *)(smem + kStatOff + 128 + par * 64);
      const double t = ((rs[0] + rs[1]) + rs[2]) + rs[3];
      uint32_t k = rk[0];
      for (int w = 1; w < 4; ++w) k = rk[w] > k ? rk[w] : k;
      g.tsum[tile] = t;
      g.tkey[tile] = k;
    };
    for (uint32_t it = 0; it <= mine; ++it) {
      if constexpr (STATS) {
        if (it >= 2 && et == 0) combine(tile_at(it - 2), (it - 2) & 1);
      }
      if (it >= 1) {
        const uint32_t prev = tile_at(it - 1);
        const uint64_t base = tile_base(prev);
        const char *ct = smem + ((it - 1) & 1) * kCtBytes;
        double st_sum = 0.0;
        int32_t st_hi = INT32_MIN, st_lo = INT32_MAX;  // signed max / min of the float bits
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const floatx4 v = *(const floatx4 *)(ct + (xlo ^ (4 * ct_swz((uint32_t)c * 1024u))));
          const uint64_t addr = base + lo + deposit_c<4, 10>((uint64_t)c, g.lpos, 4);
          floatx4 w;
#pragma unroll
          for (int e = 0; e < 4; ++e) w[e] = __builtin_amdgcn_ldexpf(v[e], sexp);
          // streaming store: the output is not read again by this kernel,
          // and keeping it out of L2 keeps the operand blocks resident
          __builtin_nontemporal_store(w, (floatx4 *)((float *)g.c0 + addr));
          if constexpr (STATS) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              st_sum += (double)w[e];
              const int32_t u = (int32_t)__float_as_uint(w[e]);
              st_hi = u > st_hi ? u : st_hi;
              st_lo = u < st_lo ? u : st_lo;
            }
          }
        }
        if constexpr (STATS) {
          // largest value: the largest non-negative pattern if there is one
          // (non-negative floats order like their signed bits), else the
          // negative pattern with the smallest signed bits; as a top-k key
          uint32_t st_k32 = st_hi >= 0 ? ((uint32_t)st_hi | 0x80000000u) : ~(uint32_t)st_lo;
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) {
            st_sum += __shfl_xor(st_sum, off);
            const uint32_t o = __shfl_xor(st_k32, off);
            st_k32 = o > st_k32 ? o : st_k32;
          }
          if (lane == 0) {
            ((double *)(smem + kStatOff + ((it - 1) & 1) * 64))[ew] = st_sum;
            ((uint32_t *)(smem + kStatOff + 128 + ((it - 1) & 1) * 64))[ew] = st_k32;
          }
        }
      }
      lds_barrier();
    }
    if constexpr (STATS) {
      if (et == 0) combine(tile_at(mine - 1), (mine - 1) & 1);
    }
  }
}

template <int P, int KP>
hipError_t launch_root_kp(const GemmArgs &g, uint32_t ntiles, int lgtn, int grid, hipStream_t s) {
  const int lgtm = g.lm - 7;
  const RootJob *none = nullptr;
  if (g.tkey)
    hipLaunchKernelGGL((root_gemm_kernel<P, KP, true, false>), dim3(grid), dim3(512), 0, s, g, ntiles, lgtm, lgtn,
                       none);
  else
    hipLaunchKernelGGL((root_gemm_kernel<P, KP, false, false>), dim3(grid), dim3(512), 0, s, g, ntiles, lgtm, lgtn,
                       none);
  return hipGetLastError();
}

template <int P, int KP>
hipError_t launch_root_multi_kp(const RootJob *jobs, int njobs, int blocks_per_job, hipStream_t s) {
  GemmArgs unused{};
  hipLaunchKernelGGL((root_gemm_kernel<P, KP, false, true>), dim3(blocks_per_job, njobs), dim3(512), 0, s, unused,
                     0u, 0, 0, jobs);
  return hipGetLastError();
}

template <int P>
hipError_t launch_root_multi_p(int kpad, const RootJob *jobs, int njobs, int blocks_per_job, hipStream_t s) {
  switch (kpad) {
    case 4:
      if constexpr (P == 1) return launch_root_multi_kp<P, 16>(jobs, njobs, blocks_per_job, s);
      return hipErrorNotSupported;
    case 5: return launch_root_multi_kp<P, 32>(jobs, njobs, blocks_per_job, s);
    case 6: return launch_root_multi_kp<P, 64>(jobs, njobs, blocks_per_job, s);
    case 7: return launch_root_multi_kp<P, 128>(jobs, njobs, blocks_per_job, s);
    case 8: return launch_root_multi_kp<P, 256>(jobs, njobs, blocks_per_job, s);
    default: return hipErrorNotSupported;
  }
}

template <int P>
hipError_t launch_root_p(const GemmArgs &g, uint32_t ntiles, int lgtn, int grid, hipStream_t s) {
  switch (g.kpad) {
    case 4:
      if constexpr (P == 1) return launch_root_kp<P, 16>(g, ntiles, lgtn, grid, s);
      return hipErrorNotSupported;
    case 5: return launch_root_kp<P, 32>(g, ntiles, lgtn, grid, s);
    case 6: return launch_root_kp<P, 64>(g, ntiles, lgtn, grid, s);
    case 7: return launch_root_kp<P, 128>(g, ntiles, lgtn, grid, s);
    case 8: return launch_root_kp<P, 256>(g, ntiles, lgtn, grid, s);
    default: return hipErrorNotSupported;
  }
}

int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace

int root_gemm_warm() { return cu_count(); }

bool root_gemm_eligible(int prec, const GemmArgs &g) {
  if (prec < 1 || prec > 4 || g.out_kind != OUT_F32) return false;
  if (g.lm < 7 || g.ln < 7 || g.lm > kMaxBits || g.ln > kMaxBits) return false;
  if (g.lm + g.ln - 14 > 30) return false;  // tile ids in 31 bits; 32 tile bits per side at most
  if (g.kpad < (prec == 1 ? 4 : 5) || g.kpad > 8 || g.lk > g.kpad) return false;
  GemmArgs h = g;
  prepare_gemm_args(h, prec, kRT, kRT);
  return h.staged && h.vec4 && h.ncompact == 14;
}

RootJob make_root_job(int prec, const GemmArgs &g_in) {
  RootJob j{};
  j.g = g_in;
  prepare_gemm_args(j.g, prec, kRT, kRT);
  j.lgtm = j.g.lm - 7;
  j.lgtn = j.g.ln - 7;
  j.ntiles = 1u << (j.lgtm + j.lgtn);
  return j;
}

hipError_t launch_root_multi(int prec, int kpad, const RootJob *jobs, int njobs, int blocks_per_job,
                             hipStream_t s) {
  if (njobs < 1 || njobs > 65535 || blocks_per_job < 8 || (blocks_per_job & 7)) return hipErrorInvalidValue;
  switch (prec) {
    case 1: return launch_root_multi_p<1>(kpad, jobs, njobs, blocks_per_job, s);
    case 2: return launch_root_multi_p<2>(kpad, jobs, njobs, blocks_per_job, s);
    case 3: return launch_root_multi_p<3>(kpad, jobs, njobs, blocks_per_job, s);
    case 4: return launch_root_multi_p<4>(kpad, jobs, njobs, blocks_per_job, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t launch_root_gemm(int prec, const GemmArgs &g_in, hipStream_t s) {
  if (!root_gemm_eligible(prec, g_in)) return hipErrorNotSupported;
  GemmArgs g = g_in;
  prepare_gemm_args(g, prec, kRT, kRT);
  // both tile counts are powers of two; tile t is (t >> lgtn, t & (2^lgtn - 1))
  const int lgtn = g.ln - 7;
  const uint32_t ntiles = 1u << (g.lm - 7 + lgtn);
  const int cus = cu_count();
  if (cus <= 0) return hipErrorNoDevice;
  const int grid = (uint32_t)cus < ntiles ? cus : (int)ntiles;
  switch (prec) {
    case 1: return launch_root_p<1>(g, ntiles, lgtn, grid, s);
    case 2: return launch_root_p<2>(g, ntiles, lgtn, grid, s);
    case 3: return launch_root_p<3>(g, ntiles, lgtn, grid, s);
    default: return launch_root_p<4>(g, ntiles, lgtn, grid, s);
  }
}

}  // namespace tqc
