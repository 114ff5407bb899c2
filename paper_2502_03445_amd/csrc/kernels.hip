// Device kernels of the contraction path: Pauli-basis transform, operand
// packing, the pairwise-contraction GEMM on CDNA4 MFMA, and the float64
// accumulator finalisation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace tqc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef double double2v __attribute__((ext_vector_type(2)));

// ======================================================= Pauli transform
// Sec. II-A: the Pauli basis of a cut is a linear combination of the
// measured / prepared variants.  Upstream end, Pauli s: the Z-basis run for
// I and Z, the X- and Y-basis runs for X and Y, summed over the measured cut
// bit with weight 1 (I) or (-1)^bit.  Downstream end: I = r0 + r1,
// Z = r0 - r1, X = 2 r+ - r0 - r1, Y = 2 ri - r0 - r1 over the preparations
// |0>, |1>, |+>, |i>.
__constant__ int kDownOpts[4] = {2, 3, 3, 2};
__constant__ int kDownPrep[4][3] = {{0, 1, 0}, {2, 0, 1}, {3, 0, 1}, {0, 1, 0}};
__constant__ double kDownCoef[4][3] = {{1, 1, 0}, {2, -1, -1}, {2, -1, -1}, {1, -1, 0}};

__global__ void __launch_bounds__(256) transform_kernel(TransformArgs a) {
  const uint64_t total = (1ull << (2 * a.c)) << a.o;
  const uint64_t cols = 1ull << (a.o + a.u);
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = e & ((1ull << a.o) - 1);
    const uint64_t row = e >> a.o;
    int sig[kMaxCutsT], nopt[kMaxCutsT], opt[kMaxCutsT];
    for (int t = 0; t < a.c; ++t) {
      sig[t] = (int)((row >> (2 * (a.c - 1 - t))) & 3);
      nopt[t] = a.up[t] ? 2 : kDownOpts[sig[t]];
      opt[t] = 0;
    }
    double sum = 0.0;
    while (true) {
      double coef = 1.0;
      uint64_t rin = 0, b = 0;
      for (int t = 0; t < a.c; ++t) {
        const int s = sig[t];
        if (a.up[t]) {
          const int meas = (s == 3) ? 0 : s;  // I and Z share the Z-basis run
          const int bit = opt[t];
          if (s != 0 && bit) coef = -coef;
          rin += (uint64_t)meas * a.w[t];
          b |= (uint64_t)bit << a.bbit[t];
        } else {
          coef *= kDownCoef[s][opt[t]];
          rin += (uint64_t)kDownPrep[s][opt[t]] * a.w[t];
        }
      }
      sum += coef * a.raw[rin * cols + ((x << a.u) | b)];
      int t = a.c - 1;
      while (t >= 0 && ++opt[t] == nopt[t]) {
        opt[t] = 0;
        --t;
      }
      if (t < 0) break;
    }
    a.out[e] = sum;
  }
}

// ================================================================= pack
__global__ void __launch_bounds__(256) pack_kernel(PackArgs a) {
  const uint64_t total = 1ull << a.nbits;
  const uint64_t kmask = (1ull << a.lk) - 1;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t src = a.base;
    for (int i = 0; i < a.nbits; ++i) src += ((e >> i) & 1ull) << a.inpos[i];
    const double v = a.src[src] * a.scale;
    const uint64_t d = ((e >> a.lk) << a.kpad) | (e & kmask);
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
}

// ============================================================= finalize
__global__ void __launch_bounds__(256) f64_to_f32_kernel(const double *in, float *out, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

__global__ void __launch_bounds__(256) scale_f64_kernel(double *buf, uint64_t n, double s) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    buf[i] *= s;
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
struct PrecTraits<3> {  // bf16x6
  using E = uint16_t;
  static constexpr int planes = 3, kgroup = 32;
  using Acc = floatx4;
};

__device__ inline uint64_t scatter_bits(uint64_t v, const uint8_t *pos, int nbits) {
  uint64_t r = 0;
  for (int i = 0; i < nbits; ++i) r |= ((v >> i) & 1ull) << pos[i];
  return r;
}

template <typename AccT>
__device__ inline void store_out(const GemmArgs &g, uint64_t addr, AccT v) {
  switch (g.out_kind) {
    case OUT_F32:
      ((float *)g.c0)[addr] = (float)((double)v * g.scale);
      break;
    case OUT_F64:
      ((double *)g.c0)[addr] = (double)v * g.scale;
      break;
    case OUT_F64_ACC:
      ((double *)g.c0)[addr] += (double)v * g.scale;
      break;
    case OUT_SPLIT2: {
      const float f = (float)((double)v * g.scale);
      const uint16_t hi = f32_to_bf16_rne(f);
      ((uint16_t *)g.c0)[addr] = hi;
      ((uint16_t *)g.c1)[addr] = f32_to_bf16_rne(f - bf16_to_f32(hi));
      break;
    }
    default: {
      const float f = (float)((double)v * g.scale);
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

template <int P, int BM, int BN, int BK>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  using T = PrecTraits<P>;
  using E = typename T::E;
  using Acc = typename T::Acc;
  constexpr int NP = T::planes;
  constexpr int ES = sizeof(E);
  constexpr int VE = 16 / ES;       // elements per 16-byte vector
  constexpr int LDR = BK + VE;      // padded LDS row (elements)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int VPR = BK / VE;      // vectors per row per plane
  constexpr int AV = BM * VPR, BV = BN * VPR;
  constexpr int AIT = (AV + 255) / 256, BIT = (BV + 255) / 256;
  static_assert(BK % T::kgroup == 0, "BK must hold whole MFMA groups");
  static_assert(FM >= 1 && FN >= 1, "tile too small");

  __shared__ __attribute__((aligned(16))) E lds[NP * (BM + BN) * LDR];
  E *As = lds;
  E *Bs = lds + NP * BM * LDR;

  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t KP = 1ull << g.kpad;
  const uint64_t tilesN = (N + BN - 1) / BN;
  const uint64_t m0 = (blockIdx.x / tilesN) * BM;
  const uint64_t n0 = (blockIdx.x % tilesN) * BN;
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

  load_global(0);
  for (uint64_t k0 = 0; k0 < KP; k0 += BK) {
    __syncthreads();
    store_lds();
    __syncthreads();
    if (k0 + BK < KP) load_global(k0 + BK);
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
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bfr[0][j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2][j], acc[i][j], 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], acc[i][j], 0, 0, 0);
          }
      }
    }
  }

  // epilogue: 16x16 block output layout.  Lane holds column lr; item r is
  // row 4*lg + r for the float32-accumulating MFMAs and row lg + 4*r for the
  // float64 MFMA (measured lane layout of v_mfma_f64_16x16x4f64).
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const uint64_t col = n0 + wn * WN + j * 16 + lr;
    if (col >= N) continue;
    const uint64_t offn = scatter_bits(col, g.posN, g.ln);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (P == 0) ? (lg + 4 * r) : (4 * lg + r);
        const uint64_t row = m0 + wm * WM + i * 16 + rr;
        if (row >= M) continue;
        const uint64_t addr = scatter_bits(row, g.posM, g.lm) + offn;
        store_out(g, addr, acc[i][j][r]);
      }
    }
  }
}

// ============================================================ launchers
static inline unsigned grid_for(uint64_t n, unsigned cap = 65536u * 4u) {
  uint64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

hipError_t launch_transform(const TransformArgs &a, hipStream_t s) {
  const uint64_t total = (1ull << (2 * a.c)) << a.o;
  hipLaunchKernelGGL(transform_kernel, dim3(grid_for(total)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(grid_for(1ull << a.nbits)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *in, float *out, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_scale_f64(double *buf, uint64_t n, double sc, hipStream_t s) {
  hipLaunchKernelGGL(scale_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, buf, n, sc);
  return hipGetLastError();
}

template <int P, int BM, int BN, int BK>
static hipError_t launch_gemm_t(const GemmArgs &g, hipStream_t s) {
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_kernel<P, BM, BN, BK>), dim3((unsigned)tiles), dim3(256), 0, s, g);
  return hipGetLastError();
}

// tile ids: 0 = 128x128, 1 = 64x64, 2 = 32x32
template <int P, int BK>
static hipError_t launch_gemm_bk(const GemmArgs &g, int tile, hipStream_t s) {
  switch (tile) {
    case 0: return launch_gemm_t<P, 128, 128, BK>(g, s);
    case 1: return launch_gemm_t<P, 64, 64, BK>(g, s);
    default: return launch_gemm_t<P, 32, 32, BK>(g, s);
  }
}

hipError_t launch_gemm(int prec, const GemmArgs &g, int tile, hipStream_t s) {
  const int kp = g.kpad;
  switch (prec) {
    case 0: return launch_gemm_bk<0, 16>(g, tile, s);
    case 1: return kp >= 5 ? launch_gemm_bk<1, 32>(g, tile, s) : launch_gemm_bk<1, 16>(g, tile, s);
    case 2: return launch_gemm_bk<2, 32>(g, tile, s);
    default: return launch_gemm_bk<3, 32>(g, tile, s);
  }
}

}  // namespace tqc
