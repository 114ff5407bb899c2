// Persistent final contraction for short K (Sec. III-B, the last pairwise
// step writes the 2^n output).
//
// The last step of a reconstruction is a GEMM with a huge M x N (the output)
// and a short K (4^c for the c cuts it closes), so its cost is storing the
// output plus the MFMA work, and both must run at once.  One workgroup per CU
// loops over 128 x 128 output tiles:
//   * operand fragments are loaded from global memory straight into the MFMA
//     register layout (no LDS), up to a whole tile ahead of their use;
//   * the accumulators of tile t are written to a staged tile in LDS (two of
//     them alternate), and the stores of tile t-1 to HBM are interleaved with
//     the MFMAs of tile t, so the store stream never waits for the math;
//   * one barrier per tile orders the staged buffers.
// Tiles are split into eight contiguous ranges, one per XCD (workgroup ids
// go round-robin over the XCDs); the workgroups of one XCD walk their range
// in row-major tile order, so the tiles in flight on an XCD share their A
// rows in its L2.  The arithmetic per accumulator is the same sequence as in
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

// OR of v over the 64 lanes of the wave (the result is wave-uniform)
__device__ inline uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

template <int P, int KP, bool STATS>
__global__ void __launch_bounds__(256) root_gemm_kernel(GemmArgs g, uint32_t ntiles, int lgtn) {
  using RT = RootTraits<P>;
  using Frag = typename RT::Frag;
  constexpr int KG = RT::KG, NP = RT::NP, ES = RT::ES;
  constexpr int NKG = KP / KG;
  constexpr int RMAX = (P == 1) ? 4 : 2;
  constexpr int R = NKG < RMAX ? NKG : RMAX;  // fragment groups in flight
  static_assert(NKG >= 1 && NKG % R == 0, "k groups");
  constexpr int FM = 4, FN = 4;  // 16 x 16 blocks per wave (64 x 64 sub-tile)

  __shared__ __attribute__((aligned(16))) char smem[kRootLds];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  // this workgroup's tiles: XCD range [r0, r1), every nslots-th from slot
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t xcd = b & 7u, slot = b >> 3;
  const uint32_t nslots = (G - xcd + 7u) >> 3;
  const uint32_t per = (ntiles + 7u) >> 3;
  const uint32_t r0 = xcd * per;
  const uint32_t r1 = r0 + per < ntiles ? r0 + per : ntiles;
  const uint32_t mine = r1 > r0 + slot ? (r1 - r0 - slot + nslots - 1) / nslots : 0;
  if (mine == 0) return;  // whole workgroup, before any barrier
  auto tile_at = [&](uint32_t i) { return r0 + slot + i * nslots; };
  const uint32_t tnmask = (1u << lgtn) - 1;

  const double scale = g.dscale ? *g.dscale : g.scale;
  const char *Ap[3] = {(const char *)g.a0, (const char *)g.a1, (const char *)g.a2};
  const char *Bp[3] = {(const char *)g.b0, (const char *)g.b1, (const char *)g.b2};

  Frag fa[R][NP][FM], fb[R][NP][FN];
  floatx4 acc[FM][FN];

  // byte offsets of this lane's first A / B fragment row of a tile
  auto a_off = [&](uint32_t tile) {
    return ((uint64_t)(tile >> lgtn) * kRT + wm * 64 + lr) * (uint64_t)(KP * ES) + 16 * lg;
  };
  auto b_off = [&](uint32_t tile) {
    return ((uint64_t)(tile & tnmask) * kRT + wn * 64 + lr) * (uint64_t)(KP * ES) + 16 * lg;
  };
  auto load_group = [&](uint64_t ao, uint64_t bo, int kg, int q) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[q][p][i] = *(const Frag *)(Ap[p] + ao + (uint64_t)(i * 16 * KP + kg * KG) * ES);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[q][p][j] = *(const Frag *)(Bp[p] + bo + (uint64_t)(j * 16 * KP + kg * KG) * ES);
    }
  };

  // tile-local row / column -> compact (output-ordered) tile index
  uint32_t tcol[FN], trow[FM][4];
#pragma unroll
  for (int j = 0; j < FN; ++j) tcol[j] = (uint32_t)deposit_c<7>(wn * 64 + j * 16 + lr, g.rankN, 7);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      trow[i][r] = (uint32_t)deposit_c<7>(wm * 64 + i * 16 + 4 * lg + r, g.rankM, 7);
  // compact index x = c * 1024 + tid * 4 + e lands at base + lo + hi(c) + e
  const uint64_t lo = deposit_c<10>((uint64_t)tid * 4, g.lpos, 10);

  double st_sum = 0.0;
  uint32_t st_k32 = 0;

  auto mfma_group = [&](int q) {
    if constexpr (P == 1) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[q][0][i][t], fb[q][0][j][t], acc[i][j], 0, 0, 0);
    } else {
      // products smallest first, the same order per accumulator as the
      // general kernel; all 16 accumulators between dependent MFMAs
      constexpr int NPR = (P == 3) ? 6 : 3;
      constexpr int pa3[6] = {2, 1, 0, 1, 0, 0}, pb3[6] = {0, 1, 2, 0, 1, 0};
      constexpr int pa2[3] = {1, 0, 0}, pb2[3] = {0, 1, 0};
#pragma unroll
      for (int pr = 0; pr < NPR; ++pr) {
        const int x = (P == 3) ? pa3[pr] : pa2[pr];
        const int y = (P == 3) ? pb3[pr] : pb2[pr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[q][x][i], fb[q][y][j], acc[i][j], 0, 0, 0);
      }
    }
  };

  auto stream_chunk = [&](const char *ct, uint64_t base, int c) {
    const uint32_t x = (uint32_t)c * 1024u + (uint32_t)tid * 4u;
    const floatx4 v = *(const floatx4 *)(ct + 4 * ct_swz(x));
    const uint64_t addr = base + lo + deposit_c<4, 10>((uint64_t)c, g.lpos, 4);
    floatx4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = (float)((double)v[e] * scale);
    *(floatx4 *)((float *)g.c0 + addr) = w;
    if constexpr (STATS) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        st_sum += (double)w[e];
        const uint32_t u = __float_as_uint(w[e]);
        const uint32_t k = u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
        st_k32 = k > st_k32 ? k : st_k32;
      }
    }
  };

  // output offset of a tile's first entry: the tile-row bits (M bits >= 7)
  // and tile-column bits deposit to their output positions; lane l handles
  // bit 7 + l of each, then the wave ORs them together
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

  // One pass: MFMAs of tile `cur` (prefetching ahead, the last groups for
  // tile `next`) interleaved with the stores of the staged tile `prev`
  // (output offset pbase).
  auto body = [&](auto MF, auto ST, uint32_t cur, uint32_t next, uint32_t prev, uint64_t pbase, int par) {
    constexpr bool DO_MF = decltype(MF)::value, DO_ST = decltype(ST)::value;
    char *ct_cur = smem + par * kCtBytes;
    const char *ct_prev = smem + (par ^ 1) * kCtBytes;
    uint64_t ca = 0, cb = 0, na = 0, nb = 0;
    if constexpr (DO_MF) {
      ca = a_off(cur);
      cb = b_off(cur);
      na = a_off(next);
      nb = b_off(next);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
    }
#pragma unroll
    for (int kg = 0; kg < NKG; ++kg) {
      if constexpr (DO_MF) {
        const int q = kg % R;
        mfma_group(q);
        if (kg + R < NKG) load_group(ca, cb, kg + R, q);
        else load_group(na, nb, kg + R - NKG, q);
      }
      if constexpr (DO_ST) {
#pragma unroll
        for (int c = kg * 16 / NKG; c < (kg + 1) * 16 / NKG; ++c) stream_chunk(ct_prev, pbase, c);
      }
    }
    if constexpr (DO_ST && STATS) {
      double s = st_sum;
      uint32_t k = st_k32;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off);
        const uint32_t o = __shfl_xor(k, off);
        k = o > k ? o : k;
      }
      if (lane == 0) {
        double *rs = (double *)(smem + kStatOff + (par ^ 1) * 64);
        uint32_t *rk = (uint32_t *)(smem + kStatOff + 128 + (par ^ 1) * 64);
        rs[wave] = s;
        rk[wave] = k;
      }
      st_sum = 0.0;
      st_k32 = 0;
    }
    if constexpr (DO_MF) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            *(float *)(ct_cur + 4 * ct_swz(trow[i][r] | tcol[j])) = acc[i][j][r];
    }
    __syncthreads();
    if constexpr (DO_ST && STATS) {
      if (tid == 0) {
        const double *rs = (const double *)(smem + kStatOff + (par ^ 1) * 64);
        const uint32_t *rk = (const uint32_t *)(smem + kStatOff + 128 + (par ^ 1) * 64);
        const double t = ((rs[0] + rs[1]) + rs[2]) + rs[3];
        uint32_t k = rk[0];
        for (int w = 1; w < 4; ++w) k = rk[w] > k ? rk[w] : k;
        g.tsum[prev] = t;
        g.tkey[prev] = k;
      }
    }
  };

  using T1 = std::true_type;
  using F0 = std::false_type;
  {
    const uint64_t ao = a_off(tile_at(0)), bo = b_off(tile_at(0));
#pragma unroll
    for (int q = 0; q < R; ++q) load_group(ao, bo, q, q);
  }
  uint64_t base = tile_base(tile_at(0));
  body(T1{}, F0{}, tile_at(0), tile_at(mine > 1 ? 1 : 0), 0, 0, 0);
  for (uint32_t i = 1; i < mine; ++i) {
    const uint64_t nbase = tile_base(tile_at(i));
    body(T1{}, T1{}, tile_at(i), tile_at(i + 1 < mine ? i + 1 : i), tile_at(i - 1), base, (int)(i & 1));
    base = nbase;
  }
  body(F0{}, T1{}, 0, 0, tile_at(mine - 1), base, (int)(mine & 1));
}

template <int P, int KP>
hipError_t launch_root_kp(const GemmArgs &g, uint32_t ntiles, int lgtn, int grid, hipStream_t s) {
  if (g.tkey)
    hipLaunchKernelGGL((root_gemm_kernel<P, KP, true>), dim3(grid), dim3(256), 0, s, g, ntiles, lgtn);
  else
    hipLaunchKernelGGL((root_gemm_kernel<P, KP, false>), dim3(grid), dim3(256), 0, s, g, ntiles, lgtn);
  return hipGetLastError();
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

bool root_gemm_eligible(int prec, const GemmArgs &g) {
  if (prec < 1 || prec > 3 || g.out_kind != OUT_F32) return false;
  if (g.lm < 7 || g.ln < 7 || g.lm > kMaxBits || g.ln > kMaxBits) return false;
  if (g.lm + g.ln - 14 > 30) return false;  // tile ids in 31 bits; 32 tile bits per side at most
  if (g.kpad < (prec == 1 ? 4 : 5) || g.kpad > 8 || g.lk > g.kpad) return false;
  GemmArgs h = g;
  prepare_gemm_args(h, prec, kRT, kRT);
  return h.staged && h.vec4 && h.ncompact == 14;
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
    default: return launch_root_p<3>(g, ntiles, lgtn, grid, s);
  }
}

}  // namespace tqc
