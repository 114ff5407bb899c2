// Device-side building blocks shared by the per-step kernels and the
// persistent batch kernel: float64 Pauli-basis transform, operand packing
// and one GEMM tile of a pairwise contraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device.hpp"

namespace tqc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// One 16x16x32 MFMA of a split form on eight 16-bit values per lane:
// bfloat16 for the bf16 forms (P = 2, 3), float16 for P = 4.
template <int P>
__device__ inline floatx4 mfma_split(const bf16x8 &a, const bf16x8 &b, const floatx4 &c) {
  if constexpr (P == 4)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
typedef double double2v __attribute__((ext_vector_type(2)));

// ======================================================= Pauli transform
// Sec. II-A: the Pauli basis of a cut is a linear combination of the
// measured / prepared variants.  Upstream end, Pauli s: the Z-basis run for
// I and Z, the X- and Y-basis runs for X and Y, summed over the measured cut
// bit with weight 1 (I) or (-1)^bit.  Downstream end: I = r0 + r1,
// Z = r0 - r1, X = 2 r+ - r0 - r1, Y = 2 ri - r0 - r1 over the preparations
// |0>, |1>, |+>, |i>.
__device__ inline int down_opts(int s) { return (s == 1 || s == 2) ? 3 : 2; }
// preparation used by option o of Pauli s: I {0,1}, X {+,0,1}, Y {i,0,1}, Z {0,1}
__device__ inline int down_prep(int s, int o) {
  if (s == 1 || s == 2) return o == 0 ? s + 1 : o - 1;
  return o;
}
__device__ inline double down_coef(int s, int o) {
  if (s == 0) return 1.0;
  if (s == 3) return o == 0 ? 1.0 : -1.0;
  return o == 0 ? 2.0 : -1.0;
}

// The options of all cuts are enumerated like an odometer (last cut
// fastest); the option digits are packed two bits per cut in a register.
__device__ inline double transform_elem(const TransformArgs &a, uint64_t e) {
  const uint64_t cols = 1ull << (a.o + a.u);
  const uint64_t x = e & ((1ull << a.o) - 1);
  const uint64_t row = e >> a.o;  // Pauli digit of cut t at bits 2 (c - 1 - t)
  uint32_t opt = 0;               // option of cut t at bits 2 t
  double sum = 0.0;
  while (true) {
    double coef = 1.0;
    uint64_t rin = 0, b = 0;
    for (int t = 0; t < a.c; ++t) {
      const int s = (int)((row >> (2 * (a.c - 1 - t))) & 3);
      const int o = (int)((opt >> (2 * t)) & 3u);
      if (a.up[t]) {
        const int meas = (s == 3) ? 0 : s;  // I and Z share the Z-basis run
        if (s != 0 && o) coef = -coef;
        rin += (uint64_t)meas * a.w[t];
        b |= (uint64_t)o << a.bbit[t];
      } else {
        coef *= down_coef(s, o);
        rin += (uint64_t)down_prep(s, o) * a.w[t];
      }
    }
    sum += coef * a.raw[rin * cols + ((x << a.u) | b)];
    int t = a.c - 1;
    for (; t >= 0; --t) {
      const int s = (int)((row >> (2 * (a.c - 1 - t))) & 3);
      const uint32_t n = a.up[t] ? 2u : (uint32_t)down_opts(s);
      const uint32_t o = ((opt >> (2 * t)) & 3u) + 1u;
      opt &= ~(3u << (2 * t));
      if (o < n) {
        opt |= o << (2 * t);
        break;
      }
    }
    if (t < 0) break;
  }
  a.out[e] = sum;
  return sum;
}

// Exponent e that brings an operand's largest |value| into [1, 2) by 2^e
// (0 for an all-zero operand); the bits are those of a non-negative double.
__device__ inline int scale_exp(unsigned long long bits) {
  const double mx = __longlong_as_double((long long)bits);
  return mx > 0.0 ? -ilogb(mx) : 0;
}

// Maximum of mx over the 256-thread workgroup, then one atomic max by its
// first thread (non-negative doubles order like their bit patterns; the
// result is not waited for).  Every thread of the workgroup calls it.
__device__ inline void amax_commit(unsigned long long *p, double mx) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(p, (unsigned long long)__double_as_longlong(m));
  }
}


// ================================================================= pack
// the power of two a leaf's values are scaled by before the cast or split
__device__ inline double pack_scale(const PackArgs &a) {
  return a.dmax ? ldexp(a.scale, scale_exp(*a.dmax)) : (a.dexp ? ldexp(a.scale, *a.dexp) : a.scale);
}

// one scaled value to destination entry d, cast or split into planes
__device__ inline void pack_store(const PackArgs &a, uint64_t d, double v) {
  switch (a.prec) {
    case 0:
      ((double *)a.dst0)[d] = v;
      break;
    case 1:
      ((float *)a.dst0)[d] = (float)v;
      break;
    case 2: {
      const uint16_t hi = f32_to_bf16_rne((float)v);
      const double r = v - (double)bf16_to_f32(hi);
      ((uint16_t *)a.dst0)[d] = hi;
      ((uint16_t *)a.dst1)[d] = f32_to_bf16_rne((float)r);
      break;
    }
    default: {
      const uint16_t hi = f32_to_bf16_rne((float)v);
      const double r1 = v - (double)bf16_to_f32(hi);
      const uint16_t mid = f32_to_bf16_rne((float)r1);
      const double r2 = r1 - (double)bf16_to_f32(mid);
      ((uint16_t *)a.dst0)[d] = hi;
      ((uint16_t *)a.dst1)[d] = mid;
      ((uint16_t *)a.dst2)[d] = f32_to_bf16_rne((float)r2);
      break;
    }
  }
}

__device__ inline void pack_elem(const PackArgs &a, uint64_t e) {
  const uint64_t kmask = (1ull << a.lk) - 1;
  uint64_t src = a.base;
  for (int i = 0; i < a.nbits; ++i) src += ((e >> i) & 1ull) << a.inpos[i];
  const double v = a.src[src] * pack_scale(a);
  pack_store(a, ((e >> a.lk) << a.kpad) | (e & kmask), v);
}

// Tiled pack, tile t of a record with tkb > 0 (2^(tkb + tsb) <= 1024
// entries; every thread of the workgroup calls it): the entries are read in
// runs of 2^tsb consecutive source entries into LDS and written in runs of
// 2^tkb consecutive destination entries (the same value per entry as
// pack_elem).
constexpr int kPackTileEntries = 1024;
__device__ inline void pack_tile(const PackArgs &a, uint64_t t, double *tile) {
  const int kb = a.tkb, sb = a.tsb, SB = 1 << sb, LD = SB + 1, n = 1 << (kb + sb);
  const uint64_t kmask = (1ull << a.lk) - 1;
  // the tile's fixed destination-index bits: t deposited into tmask
  uint64_t e0 = 0, src0 = a.base;
  {
    uint64_t tt = t;
    for (int j = 0; j < a.nbits && tt; ++j)
      if ((a.tmask >> j) & 1ull) {
        if (tt & 1ull) {
          e0 |= 1ull << j;
          src0 += 1ull << a.inpos[j];
        }
        tt >>= 1;
      }
  }
  const uint64_t d0 = ((e0 >> a.lk) << a.kpad) | (e0 & kmask);
  const double sc = pack_scale(a);
  // reads: source bits 0..sb-1 fastest
  for (int l = (int)threadIdx.x; l < n; l += (int)blockDim.x) {
    const int s = l & (SB - 1), kk = l >> sb;
    uint64_t src = src0 + (uint64_t)s;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < kb) src += (uint64_t)((kk >> i) & 1) << a.inpos[i];
    tile[kk * LD + s] = a.src[src] * sc;
  }
  __syncthreads();
  // writes: destination bits 0..kb-1 (the k bits) fastest
  for (int l = (int)threadIdx.x; l < n; l += (int)blockDim.x) {
    const int kk = l & ((1 << kb) - 1), s = l >> kb;
    uint64_t d = d0 + (uint64_t)kk;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < sb) d += (uint64_t)((s >> q) & 1) << a.dpos[q];
    pack_store(a, d, tile[kk * LD + s]);
  }
  __syncthreads();  // the tile is free for the workgroup's next one
}

__device__ inline double gathered_abs(const AbsMaxArgs &a, uint64_t e) {
  uint64_t src = a.base;
  for (int i = 0; i < a.nbits; ++i) src += ((e >> i) & 1ull) << a.inpos[i];
  return fabs(a.src[src]);
}

// ================================================================= GEMM
// One pairwise contraction C[m][n] = sum_k A[m][k] B[n][k] (Sec. III-B): the
// shared cut digits are k, each operand's other index bits are m or n, and
// both operands are stored as row-major [rows][2^kpad] with k contiguous.
// The result is scattered to its consumer's layout: bit i of m lands on
// output bit posM[i] (likewise for n), so the final step writes the
// probability vector in qubit order and earlier steps write the next
// step's operand directly.
//
// Block: 256 threads = 4 waves in a 2x2 arrangement; each wave owns a
// (BM/2) x (BN/2) sub-tile built from 16x16 MFMA blocks.  The k index inside
// an MFMA group is remapped so that every lane fetches one contiguous
// 16-byte run of its row from LDS: lane group g (= lane / 16) at step t
// holds logical k = 4g + t (fp32/fp64, 16 k per group) or k = 8g + e
// (bfloat16, 32 k per group).
template <int P>
struct PrecTraits;
template <>
struct PrecTraits<0> {  // float64
  using E = double;
  static constexpr int planes = 1, kgroup = 16;
  using Acc = doublex4;
};
template <>
struct PrecTraits<1> {  // float32
  using E = float;
  static constexpr int planes = 1, kgroup = 16;
  using Acc = floatx4;
};
template <>
struct PrecTraits<2> {  // bf16x3
  using E = uint16_t;
  static constexpr int planes = 2, kgroup = 32;
  using Acc = floatx4;
};
template <>
struct PrecTraits<4> {  // fp16x3 (final step of a float16-split plan)
  using E = uint16_t;
  static constexpr int planes = 2, kgroup = 32;
  using Acc = floatx4;
};
template <>
struct PrecTraits<3> {  // bf16x6
  using E = uint16_t;
  static constexpr int planes = 3, kgroup = 32;
  using Acc = floatx4;
};

// Bit deposit with a compile-time bound: every pos[] index is a constant, so
// the positions are loaded once (scalar) instead of once per bit and lane.
template <int MAXB, int OFF = 0, typename A>
__device__ inline uint64_t deposit_c(uint64_t v, const A &pos, int nbits) {
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < MAXB; ++i)
    if (i < nbits) r |= ((v >> i) & 1ull) << pos[OFF + i];
  return r;
}

__device__ inline uint64_t scatter_bits(uint64_t v, const uint8_t *pos, int nbits) {
  uint64_t r = 0;
  for (int i = 0; i < nbits; ++i) r |= ((v >> i) & 1ull) << pos[i];
  return r;
}

template <typename AccT>
__device__ inline void store_out(const GemmArgs &g, double scale, uint64_t addr, AccT v) {
  switch (g.out_kind) {
    case OUT_F32:
      ((float *)g.c0)[addr] = (float)((double)v * scale);
      break;
    case OUT_F64:
      ((double *)g.c0)[addr] = (double)v * scale;
      break;
    case OUT_F64_ACC:
      ((double *)g.c0)[addr] += (double)v * scale;
      break;
    case OUT_SPLIT2: {
      const float f = (float)((double)v * scale);
      const uint16_t hi = f32_to_bf16_rne(f);
      ((uint16_t *)g.c0)[addr] = hi;
      ((uint16_t *)g.c1)[addr] = f32_to_bf16_rne(f - bf16_to_f32(hi));
      break;
    }
    default: {
      const float f = (float)((double)v * scale);
      const uint16_t hi = f32_to_bf16_rne(f);
      const float r1 = f - bf16_to_f32(hi);
      const uint16_t mid = f32_to_bf16_rne(r1);
      ((uint16_t *)g.c0)[addr] = hi;
      ((uint16_t *)g.c1)[addr] = mid;
      ((uint16_t *)g.c2)[addr] = f32_to_bf16_rne(r1 - bf16_to_f32(mid));
      break;
    }
  }
}

// Tile order: with 8 XCDs, consecutive workgroup ids go round-robin to the
// XCDs.  Remap so that each XCD owns a contiguous eighth of the tile space and
// walks it in groups of 8 tile rows (A row-blocks) by increasing column:
// the tiles resident on one XCD at a time share A and B blocks in its L2.
__device__ inline void tile_of(uint64_t bid, uint64_t tilesM, uint64_t tilesN, int swz,
                               uint64_t &tm, uint64_t &tn) {
  const uint64_t T = tilesM * tilesN;
  uint64_t t = bid;
  if (swz) {
    const uint64_t per = T >> 3;
    t = (bid & 7) * per + (bid >> 3);
    const uint64_t G = 8;
    const uint64_t grp = t / (G * tilesN);
    const uint64_t r = t % (G * tilesN);
    tm = grp * G + (r % G);
    tn = r / G;
    return;
  }
  tm = t / tilesN;
  tn = t % tilesN;
}

__device__ inline uint32_t deposit(uint32_t v, const uint8_t *pos, int nbits) {
  uint32_t r = 0;
  for (int i = 0; i < nbits; ++i) r |= ((v >> i) & 1u) << pos[i];
  return r;
}

template <int P, int BM, int BN, int BK>
struct GemmShape {
  using T = PrecTraits<P>;
  using E = typename T::E;
  static constexpr int NP = T::planes;
  static constexpr int ES = sizeof(E);
  static constexpr int VE = 16 / ES;
  static constexpr int LDR = BK + VE;
  static constexpr int OPER_BYTES = NP * (BM + BN) * LDR * ES;
  static constexpr int CT_BYTES = (P == 0) ? 0 : BM * BN * 4;  // staged float tile
  static constexpr int MAIN_BYTES = OPER_BYTES > CT_BYTES ? OPER_BYTES : CT_BYTES;
  static constexpr int STAT_OFF = MAIN_BYTES;  // 4 waves x (sum, key) of the tile statistics
  static constexpr int LDS_BYTES = MAIN_BYTES + 64;
};

// order-preserving unsigned keys of stored output values (larger value,
// larger key); the float32 key is the one the top-k kernels use
__device__ inline uint64_t out_key_f32(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? (uint64_t)(~u) : (uint64_t)(u | 0x80000000u);
}
__device__ inline uint64_t out_key_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// Epilogue of one output tile (shared by the GEMM kernels): result(i, j, r)
// is item r of 16x16 block (i, j) of the calling wave as a double.  Stores
// the scaled tile in the consumer's layout (staged through LDS in output
// order when `staged`), the split-k partials, or scatters directly; writes
// the tile statistics when the step asks for them.  `smem` holds at least
// the staged float tile, and `stat_off` 64 bytes for the statistics.
template <int P, int BM, int BN, typename R>
__device__ __attribute__((always_inline)) inline void gemm_epilogue(const GemmArgs &g, char *smem, int stat_off,
                                                                     uint64_t tm, uint64_t tn, uint64_t split,
                                                                     bool staged, R result) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t tilesN = (N + BN - 1) / BN;
  const uint64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const double scale = g.dscale ? *g.dscale : g.scale;
  // tile statistics of the stored values (float32 / float64 outputs only)
  const bool want_stats = g.tkey != nullptr;
  double st_sum = 0.0;
  uint64_t st_key = 0;
  uint32_t st_k32 = 0;
  auto note = [&](double y) {  // y = accumulator * scale, before the store's rounding
    if (g.out_kind == OUT_F32) {
      const float f = (float)y;
      st_sum += (double)f;
      const uint32_t u = __float_as_uint(f);
      const uint32_t k = u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);  // out_key_f32
      st_k32 = k > st_k32 ? k : st_k32;
    } else {
      st_sum += y;
      const uint64_t k = out_key_f64(y);
      st_key = k > st_key ? k : st_key;
    }
  };
  auto finish_stats = [&]() {
    if (g.out_kind == OUT_F32) st_key = st_k32;
    // fixed-order reduction: lanes by xor butterfly, then waves 0..3
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      st_sum += __shfl_xor(st_sum, off);
      const uint64_t o = __shfl_xor(st_key, off);
      st_key = o > st_key ? o : st_key;
    }
    double *rs = (double *)(smem + stat_off);
    uint64_t *rk = (uint64_t *)(smem + stat_off + 32);
    if (lane == 0) {
      rs[wave] = st_sum;
      rk[wave] = st_key;
    }
    __syncthreads();
    if (tid == 0) {
      const double t = ((rs[0] + rs[1]) + rs[2]) + rs[3];
      uint64_t k = rk[0];
      for (int w = 1; w < 4; ++w) k = rk[w] > k ? rk[w] : k;
      g.tsum[tm * tilesN + tn] = t;
      g.tkey[tm * tilesN + tn] = k;
    }
  };
  // Epilogue.  16x16 block output layout: lane holds column lr; item r is row
  // 4*lg + r for the float32-accumulating MFMAs and row lg + 4*r for the
  // float64 MFMA (measured lane layout of v_mfma_f64_16x16x4f64).
  if (staged) {
    // 1) accumulators -> LDS at their compact (output-order) tile index,
    //    16-byte chunks XOR-swizzled by higher index bits so that the
    //    scattered single-float writes spread over the LDS banks; float4
    //    reads at multiples of 4 stay contiguous
    float *ct = (float *)smem;
    auto swz = [](uint32_t c) { return c ^ ((((c >> 5) ^ (c >> 8) ^ (c >> 11)) & 7u) << 2); };
    __syncthreads();  // operand tiles no longer needed
    constexpr int LBM = __builtin_ctz(BM), LBN = __builtin_ctz(BN);
    uint32_t tcol[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) tcol[j] = (uint32_t)deposit_c<LBN>(wn * WN + j * 16 + lr, g.rankN, LBN);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t trow = (uint32_t)deposit_c<LBM>(wm * WM + i * 16 + 4 * lg + r, g.rankM, LBM);
#pragma unroll
        for (int j = 0; j < FN; ++j) ct[swz(trow | tcol[j])] = (float)result(i, j, r);
      }
    __syncthreads();
    // 2) stream the tile out in output order: compact index x maps to the
    //    output offset sum_b bit_b(x) << lpos[b]; the bits below the stride
    //    of the loop are fixed per thread
    const uint64_t base = deposit_c<kMaxBits>(m0, g.posM, g.lm) + deposit_c<kMaxBits>(n0, g.posN, g.ln);
    constexpr int TT = BM * BN;
    constexpr int NCB = LBM + LBN;
    if (g.vec4) {
      constexpr int LB = 10;  // log2(256 threads * 4)
      const uint64_t lo = deposit_c<LB>((uint64_t)tid * 4, g.lpos, LB);
#pragma unroll 4
      for (int it = 0; it * 1024 < TT; ++it) {
        const int x = it * 1024 + tid * 4;
        const uint64_t addr = base + lo + deposit_c<(NCB > LB ? NCB - LB : 1), LB>((uint64_t)it, g.lpos, NCB - LB);
        const floatx4 v = *(const floatx4 *)(ct + swz((uint32_t)x));
        switch (g.out_kind) {
          case OUT_F32: {
            floatx4 w;
#pragma unroll
            for (int e = 0; e < 4; ++e) w[e] = (float)((double)v[e] * scale);
            *(floatx4 *)((float *)g.c0 + addr) = w;
            if (want_stats)
#pragma unroll
              for (int e = 0; e < 4; ++e) note((double)v[e] * scale);
            break;
          }
          case OUT_F64_ACC: {
            double *o = (double *)g.c0 + addr;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] += (double)v[e] * scale;
            break;
          }
          case OUT_F64: {
            double *o = (double *)g.c0 + addr;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (double)v[e] * scale;
            if (want_stats)
#pragma unroll
              for (int e = 0; e < 4; ++e) note((double)v[e] * scale);
            break;
          }
          case OUT_SPLIT2:
          case OUT_SPLIT3: {
            // the next step's bfloat16 planes: the four values of each plane
            // in one 8-byte store (addr is a multiple of 4 here), so a
            // wave's store covers whole lines
            uint32_t h[2] = {0, 0}, m[2] = {0, 0}, l[2] = {0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float f = (float)((double)v[e] * scale);
              const uint16_t hi = f32_to_bf16_rne(f);
              const float r1 = f - bf16_to_f32(hi);
              const uint16_t b1 = f32_to_bf16_rne(r1);
              h[e >> 1] |= (uint32_t)hi << (16 * (e & 1));
              m[e >> 1] |= (uint32_t)b1 << (16 * (e & 1));
              if (g.out_kind == OUT_SPLIT3)
                l[e >> 1] |= (uint32_t)f32_to_bf16_rne(r1 - bf16_to_f32(b1)) << (16 * (e & 1));
            }
            *(uint2 *)((uint16_t *)g.c0 + addr) = uint2{h[0], h[1]};
            *(uint2 *)((uint16_t *)g.c1 + addr) = uint2{m[0], m[1]};
            if (g.out_kind == OUT_SPLIT3) *(uint2 *)((uint16_t *)g.c2 + addr) = uint2{l[0], l[1]};
            break;
          }
          default: {
#pragma unroll
            for (int e = 0; e < 4; ++e) store_out(g, scale, addr + e, v[e]);
            break;
          }
        }
      }
    } else {
      constexpr int LB = 8;  // log2(256 threads)
      const uint64_t lo = deposit_c<LB>((uint64_t)tid, g.lpos, LB);
      for (int it = 0; it * 256 < TT; ++it) {
        const uint64_t addr = base + lo + deposit_c<(NCB > LB ? NCB - LB : 1), LB>((uint64_t)it, g.lpos, NCB - LB);
        const float v = ct[swz((uint32_t)(it * 256 + tid))];
        store_out(g, scale, addr, v);
        if (want_stats) note((double)v * scale);
      }
    }
    if (want_stats) finish_stats();
    return;
  }
  // split-K partial results: unscaled float64, dense [split][m][n]
  if (g.ksplit) {
    double *part = g.partial + split * M * N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (P == 0) ? (lg + 4 * r) : (4 * lg + r);
        const uint64_t row = m0 + wm * WM + i * 16 + rr;
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const uint64_t col = n0 + wn * WN + j * 16 + lr;
          if (col < N) part[row * N + col] = result(i, j, r);
        }
      }
    return;
  }
  // direct scatter (partial tiles, float64 form): row = m0 | local row, the
  // tile base and the tile-local bits deposit separately
  {
    constexpr int LBM = __builtin_ctz(BM), LBN = __builtin_ctz(BN);
    const int lbm = g.lm < LBM ? g.lm : LBM, lbn = g.ln < LBN ? g.ln : LBN;
    const uint64_t basem = deposit_c<kMaxBits>(m0, g.posM, g.lm);
    const uint64_t basen = deposit_c<kMaxBits>(n0, g.posN, g.ln);
    uint64_t offn[FN];
    bool okn[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int cl = wn * WN + j * 16 + lr;
      okn[j] = n0 + cl < N;
      offn[j] = basen + deposit_c<LBN>((uint64_t)cl, g.posN, lbn);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (P == 0) ? (lg + 4 * r) : (4 * lg + r);
        const int rl = wm * WM + i * 16 + rr;
        if (m0 + rl >= M) continue;
        const uint64_t offm = basem + deposit_c<LBM>((uint64_t)rl, g.posM, lbm);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          if (okn[j]) {
            const double v = result(i, j, r);
            store_out(g, scale, offm + offn[j], v);
            if (want_stats) note(v * scale);
          }
      }
    }
  }
  if (want_stats) finish_stats();
}

// A64: float32 MFMA sums over 256-long k chunks are folded into float64
// accumulators (long float32 chains would exceed 1e-6 relative error).
template <int P, int BM, int BN, int BK, bool A64 = false>
__device__ __attribute__((always_inline)) inline void gemm_tile(const GemmArgs &g, uint64_t bid, char *smem) {
  using T = PrecTraits<P>;
  using E = typename T::E;
  using Acc = typename T::Acc;
  using S = GemmShape<P, BM, BN, BK>;
  constexpr int NP = T::planes;
  constexpr int VE = S::VE;
  constexpr int LDR = S::LDR;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int VPR = BK / VE;      // vectors per row per plane
  constexpr int AV = BM * VPR, BV = BN * VPR;
  constexpr int AIT = (AV + 255) / 256, BIT = (BV + 255) / 256;
  static_assert(BK % T::kgroup == 0, "BK must hold whole MFMA groups");
  static_assert(FM >= 1 && FN >= 1, "tile too small");

  E *As = (E *)smem;
  E *Bs = As + NP * BM * LDR;

  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t KP = 1ull << g.kpad;
  const uint64_t tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  // split-K: the low bits of the workgroup id pick the k range
  const uint64_t split = g.ksplit ? (bid & ((1ull << g.ksplit) - 1)) : 0;
  if (g.ksplit) bid >>= g.ksplit;
  const uint64_t klen = KP >> g.ksplit, kbeg = split * klen, kend = kbeg + klen;
  uint64_t tm, tn;
  tile_of(bid, tilesM, tilesN, g.swz, tm, tn);
  const uint64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

  const E *Ap[3] = {(const E *)g.a0, (const E *)g.a1, (const E *)g.a2};
  const E *Bp[3] = {(const E *)g.b0, (const E *)g.b1, (const E *)g.b2};

  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};
  constexpr int AM = A64 ? FM : 1, AN = A64 ? FN : 1;
  doublex4 acc2[AM][AN];
#pragma unroll
  for (int i = 0; i < AM; ++i)
#pragma unroll
    for (int j = 0; j < AN; ++j) acc2[i][j] = doublex4{0, 0, 0, 0};

  uint4 ra[NP][AIT], rb[NP][BIT];
  auto load_global = [&](uint64_t k0) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int v = tid + it * 256;
        uint4 val = {0, 0, 0, 0};
        if (v < AV) {
          const int r = v / VPR, cv = v % VPR;
          const uint64_t row = m0 + r;
          if (row < M) val = *(const uint4 *)(Ap[p] + row * KP + k0 + cv * VE);
        }
        ra[p][it] = val;
      }
#pragma unroll
      for (int it = 0; it < BIT; ++it) {
        const int v = tid + it * 256;
        uint4 val = {0, 0, 0, 0};
        if (v < BV) {
          const int r = v / VPR, cv = v % VPR;
          const uint64_t row = n0 + r;
          if (row < N) val = *(const uint4 *)(Bp[p] + row * KP + k0 + cv * VE);
        }
        rb[p][it] = val;
      }
    }
  };
  auto store_lds = [&]() {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int v = tid + it * 256;
        if (v < AV) {
          const int r = v / VPR, cv = v % VPR;
          *(uint4 *)(As + (p * BM + r) * LDR + cv * VE) = ra[p][it];
        }
      }
#pragma unroll
      for (int it = 0; it < BIT; ++it) {
        const int v = tid + it * 256;
        if (v < BV) {
          const int r = v / VPR, cv = v % VPR;
          *(uint4 *)(Bs + (p * BN + r) * LDR + cv * VE) = rb[p][it];
        }
      }
    }
  };

  // float64 results (A64 with a float64 output) skip the float staging
  const bool staged = (P != 0) && g.staged && !g.ksplit &&
                      (!A64 || (g.out_kind != OUT_F64 && g.out_kind != OUT_F64_ACC));

  load_global(kbeg);
  for (uint64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    store_lds();
    __syncthreads();
    if (k0 + BK < kend) load_global(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += T::kgroup) {
      if constexpr (P == 0 || P == 1) {
        using V4 = typename std::conditional<P == 0, doublex4, floatx4>::type;
        V4 af[FM], bfr[FN];
        // rows are 16-byte aligned in LDS: read 16-byte pieces
        auto rd = [](const E *ptr) -> V4 {
          if constexpr (P == 0) {
            const double2v lo = *(const double2v *)ptr;
            const double2v hi = *(const double2v *)(ptr + 2);
            return V4{lo[0], lo[1], hi[0], hi[1]};
          } else {
            return *(const V4 *)ptr;
          }
        };
#pragma unroll
        for (int i = 0; i < FM; ++i) af[i] = rd(As + (wm * WM + i * 16 + lr) * LDR + kk + 4 * lg);
#pragma unroll
        for (int j = 0; j < FN; ++j) bfr[j] = rd(Bs + (wn * WN + j * 16 + lr) * LDR + kk + 4 * lg);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
              if constexpr (P == 0)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][t], bfr[j][t], acc[i][j], 0, 0, 0);
              else
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][t], bfr[j][t], acc[i][j], 0, 0, 0);
            }
      } else {
        bf16x8 af[NP][FM], bfr[NP][FN];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
            af[p][i] = *(const bf16x8 *)(As + (p * BM + wm * WM + i * 16 + lr) * LDR + kk + 8 * lg);
#pragma unroll
          for (int j = 0; j < FN; ++j)
            bfr[p][j] = *(const bf16x8 *)(Bs + (p * BN + wn * WN + j * 16 + lr) * LDR + kk + 8 * lg);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            // small terms first, then the leading product
            if constexpr (P == 3) {
              acc[i][j] = mfma_split<P>(af[2][i], bfr[0][j], acc[i][j]);
              acc[i][j] = mfma_split<P>(af[1][i], bfr[1][j], acc[i][j]);
              acc[i][j] = mfma_split<P>(af[0][i], bfr[2][j], acc[i][j]);
            }
            acc[i][j] = mfma_split<P>(af[1][i], bfr[0][j], acc[i][j]);
            acc[i][j] = mfma_split<P>(af[0][i], bfr[1][j], acc[i][j]);
            acc[i][j] = mfma_split<P>(af[0][i], bfr[0][j], acc[i][j]);
          }
      }
    }
    if constexpr (A64 && P != 0) {
      if (((k0 + BK) & 255) == 0 || k0 + BK >= kend) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc2[i][j][r] += (double)acc[i][j][r];
            acc[i][j] = Acc{0, 0, 0, 0};
          }
      }
    }
  }
  auto result = [&](int i, int j, int r) -> double {
    if constexpr (A64 && P != 0) return acc2[i][j][r];
    else return (double)acc[i][j][r];
  };

  gemm_epilogue<P, BM, BN>(g, smem, S::STAT_OFF, tm, tn, split, staged, result);
}

// Tile-dependent epilogue parameters (host side): the tile's output bits in
// increasing order define the compact index used to stage C through LDS.
inline void prepare_gemm_args(GemmArgs &g, int prec, int BM, int BN) {
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  const uint64_t tiles = tilesM * tilesN;
  const int P = prec;
  const int bm = __builtin_ctz(BM), bn = __builtin_ctz(BN);
  g.staged = 0;
  g.vec4 = 0;
  g.swz = (tiles >= 64 && tilesM >= 8 && (tiles % 64) == 0) ? 1 : 0;
  if (P != 0 && g.lm >= bm && g.ln >= bn) {
    // compact tile index: the tile's output bits in increasing order
    int pos[32], n = 0;
    for (int i = 0; i < bm; ++i) pos[n++] = g.posM[i];
    for (int j = 0; j < bn; ++j) pos[n++] = g.posN[j];
    for (int a = 1; a < n; ++a)
      for (int b = a; b > 0 && pos[b - 1] > pos[b]; --b) {
        const int t = pos[b];
        pos[b] = pos[b - 1];
        pos[b - 1] = t;
      }
    for (int b = 0; b < n; ++b) g.lpos[b] = (uint8_t)pos[b];
    auto rank = [&](int p) {
      for (int b = 0; b < n; ++b)
        if (pos[b] == p) return b;
      return -1;
    };
    for (int i = 0; i < bm; ++i) g.rankM[i] = (uint8_t)rank(g.posM[i]);
    for (int j = 0; j < bn; ++j) g.rankN[j] = (uint8_t)rank(g.posN[j]);
    g.ncompact = n;
    g.vec4 = (n >= 10 && pos[0] == 0 && pos[1] == 1) ? 1 : 0;
    g.staged = (n <= 16 && n >= 8) ? 1 : 0;
  }
}

inline int tile_bm(int tile) { return tile == 0 ? 128 : (tile == 1 ? 64 : 32); }

}  // namespace tqc
