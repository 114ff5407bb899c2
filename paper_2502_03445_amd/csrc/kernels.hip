// Kernels of the contraction path (one launch per pass or step): Pauli-basis
// transform, operand packing, pairwise-contraction GEMM, float64 finalize.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_ops.hpp"
#include "kernels.hpp"

namespace tqc {

// abs-max of a transform's written entry e (fixed-qubit filter)
template <typename A>
__device__ inline void amax_take(const A &a, uint64_t e, double v, double &mx) {
  if ((e & a.amask) == a.abase) mx = fmax(mx, fabs(v));
}

__device__ inline void transform_range(const TransformArgs &a, uint64_t e0, uint64_t step) {
  const uint64_t total = (1ull << (2 * a.c)) << a.o;
  double mx = 0.0;
  for (uint64_t e = e0; e < total; e += step) {
    const double v = transform_elem(a, e);
    if (a.amax) amax_take(a, e, v, mx);
  }
  if (a.amax) amax_commit(a.amax, mx);
}

__global__ void __launch_bounds__(256) transform_kernel(TransformArgs a) {
  transform_range(a, blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}

// several tensors per launch (blockIdx.y selects the tensor)
struct TransformBatch {
  TransformArgs a[4];
};
__global__ void __launch_bounds__(256) transform_multi_kernel(TransformBatch tb) {
  transform_range(tb.a[blockIdx.y], blockIdx.x * (uint64_t)blockDim.x + threadIdx.x,
                  (uint64_t)gridDim.x * blockDim.x);
}

__global__ void __launch_bounds__(256) pack_kernel(PackArgs a) {
  const uint64_t total = 1ull << a.nbits;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    pack_elem(a, e);
}

// several leaf operands per launch (blockIdx.y selects the leaf)
struct PackBatch {
  PackArgs a[kPackBatch];
  uint32_t nblk[kPackBatch];  // workgroups of each leaf (the first ones of its row)
  ScaleRec sr;                // optional (maxbits non-null): exponents and output scale
};
__device__ inline void write_scales(const ScaleRec &q);

// workgroup b of nb for one leaf: tiles b, b + nb, ... or entries
// grid-stride (every thread of the workgroup calls it)
__device__ inline void pack_range(const PackArgs &a, uint64_t b, uint64_t nb, double *tile) {
  if (a.tkb > 0) {
    const uint64_t tiles = 1ull << (a.nbits - a.tkb - a.tsb);
    for (uint64_t t = b; t < tiles; t += nb) pack_tile(a, t, tile);
    return;
  }
  const uint64_t total = 1ull << a.nbits;
  for (uint64_t e = b * blockDim.x + threadIdx.x; e < total; e += nb * blockDim.x) pack_elem(a, e);
}

__global__ void __launch_bounds__(256) pack_multi_kernel(PackBatch pb) {
  __shared__ double tile[kPackTileEntries + 32];
  if (pb.sr.maxbits && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) write_scales(pb.sr);
  const uint32_t nb = pb.nblk[blockIdx.y];
  if (blockIdx.x >= nb) return;  // whole workgroup
  pack_range(pb.a[blockIdx.y], blockIdx.x, nb, tile);
}

__global__ void __launch_bounds__(256) f64_to_f32_kernel(const double *in, float *out, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// zero fill (a kernel rather than a memset node, so it can be captured in a
// graph and replayed)
__global__ void __launch_bounds__(256) zero_u64_kernel(unsigned long long *buf, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    buf[i] = 0ull;
}

__global__ void __launch_bounds__(256) scale_f64_kernel(double *buf, uint64_t n, double s) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    buf[i] *= s;
}

// several leaves per launch (blockIdx.y selects the leaf)
struct AbsMaxBatch {
  AbsMaxArgs a[kPackBatch];
};
__global__ void __launch_bounds__(256) absmax_kernel(AbsMaxBatch ab) {
  const AbsMaxArgs &a = ab.a[blockIdx.y];
  __shared__ double red[256];
  const uint64_t total = 1ull << a.nbits;
  double mx = 0.0;
#pragma unroll 4
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    mx = fmax(mx, gathered_abs(a, e));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(a.out, (unsigned long long)__double_as_longlong(red[0]));
}

// exponents e_j = -floor(log2 max_j) (0 for an all-zero operand) and the
// output scale 2^(-K - sum e_j)
__device__ inline void write_scales(const ScaleRec &q) {
  int sum = 0;
  for (int j = 0; j < q.m; ++j) {
    const int e = scale_exp(q.maxbits[j]);
    q.exps[j] = e;
    sum += e;
  }
  *q.root_scale = ldexp(1.0, -q.K - sum);
}

// split-K reduction: entry e = m * N + n adds its 2^ksplit partial sums in
// split order (float64), then stores like the GEMM epilogue
__global__ void __launch_bounds__(256) splitk_reduce_kernel(GemmArgs g) {
  const uint64_t MN = 1ull << (g.lm + g.ln);
  const int S = 1 << g.ksplit;
  const double scale = g.dscale ? *g.dscale : g.scale;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < MN;
       e += (uint64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int sp = 0; sp < S; ++sp) v += g.partial[sp * MN + e];
    const uint64_t addr = scatter_bits(e >> g.ln, g.posM, g.lm) + scatter_bits(e & ((1ull << g.ln) - 1), g.posN, g.ln);
    store_out(g, scale, addr, v);
  }
}

template <int P, int BM, int BN, int BK, bool A64>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) char smem[GemmShape<P, BM, BN, BK>::LDS_BYTES];
  gemm_tile<P, BM, BN, BK, A64>(g, blockIdx.x, smem);
}

// ============================================================ launchers
// Reductions that end in one atomic per workgroup on a single address keep
// their grids at one workgroup per CU: those atomics serialize (about 26 ns
// each measured here), so 1024 workgroups spend ~27 us on them alone.
constexpr unsigned kMaxGrid = 256;

static inline unsigned grid_for(uint64_t n, unsigned cap = 65536u * 4u);

// Workgroups of a leaf's pack: one per tile when tiled, else one entry per
// thread.
static inline unsigned pack_blocks(const PackArgs &a) {
  if (a.tkb > 0) return grid_for((1ull << (a.nbits - a.tkb - a.tsb)) * 256);
  return grid_for(1ull << a.nbits);
}

// Workgroups of a transform record (one entry or free coordinate per
// thread, grid-stride beyond): one that also takes an abs-max ends in one
// atomic per workgroup on the leaf's address, and such atomics serialize
// (about 26 ns each), so its grid stops at 1024 workgroups.
constexpr unsigned kAmaxGrid = 1024;
static inline unsigned transform_grid(uint64_t n, bool amax) {
  const unsigned g = grid_for(n);
  return amax && g > kAmaxGrid ? kAmaxGrid : g;
}

static inline unsigned grid_for(uint64_t n, unsigned cap) {
  uint64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

// Separable transform pass (Sec. II-A maps, one cut at a time).  Downstream
// end, preparations |0>, |1>, |+>, |i>: I = r0 + r1, X = 2 r+ - r0 - r1,
// Y = 2 ri - r0 - r1, Z = r0 - r1.  Upstream end, bases Z, X, Y with
// measured bit b: I = Z0 + Z1, X = X0 - X1, Y = Y0 - Y1, Z = Z0 - Z1.
__device__ inline void down_map(const double r[4], double p[4]) {
  const double s01 = r[0] + r[1];
  p[0] = s01;
  p[1] = 2.0 * r[2] - s01;
  p[2] = 2.0 * r[3] - s01;
  p[3] = r[0] - r[1];
}
__device__ inline void up_map(const double v[6], double p[4]) {
  p[0] = v[0] + v[1];
  p[1] = v[2] - v[3];
  p[2] = v[4] - v[5];
  p[3] = v[0] - v[1];
}

template <bool UP>
__device__ inline uint64_t variant_off(const TransformPassArgs &a, int i, int v) {
  if constexpr (UP) return (uint64_t)(v >> 1) * a.row_in[i] + (uint64_t)(v & 1) * a.bit_in[i];
  else return (uint64_t)v * a.row_in[i];
}

template <bool UP>
__device__ inline void cut_map(const double *v, double *p) {
  if constexpr (UP) up_map(v, p);
  else down_map(v, p);
}

// One thread per free coordinate: loads every variant of the pass cuts,
// applies the first cut's map then the second's, stores 4 or 16 digits.
// Consecutive threads take consecutive innermost coordinates, so every
// load and store instruction of a wave covers consecutive addresses.
template <int G, bool UA, bool UB>
__device__ inline void pass_body(const TransformPassArgs &a, uint64_t bid, uint64_t nblk) {
  constexpr int NA = UA ? 6 : 4;
  constexpr int NB = G == 2 ? (UB ? 6 : 4) : 1;
  const uint64_t stride = nblk * blockDim.x;
  const bool small = a.nfree <= 0xffffffffull;
  double mx = 0.0;
  for (uint64_t f = bid * blockDim.x + threadIdx.x; f < a.nfree; f += stride) {
    uint64_t ib = 0, ob = 0;
    if (small) {
      uint32_t r = (uint32_t)f;
      for (int s = 0; s < a.nseg - 1; ++s) {
        const uint32_t e = (uint32_t)a.seg_ext[s];
        const uint32_t q = r / e, c = r - q * e;
        ib += (uint64_t)c * a.seg_in[s];
        ob += (uint64_t)c * a.seg_out[s];
        r = q;
      }
      ib += (uint64_t)r * a.seg_in[a.nseg - 1];
      ob += (uint64_t)r * a.seg_out[a.nseg - 1];
    } else {
      uint64_t r = f;
      for (int s = 0; s < a.nseg - 1; ++s) {
        const uint64_t e = a.seg_ext[s];
        const uint64_t q = r / e, c = r - q * e;
        ib += c * a.seg_in[s];
        ob += c * a.seg_out[s];
        r = q;
      }
      ib += r * a.seg_in[a.nseg - 1];
      ob += r * a.seg_out[a.nseg - 1];
    }
    double v[NA * NB];
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        uint64_t off = ib + variant_off<UA>(a, 0, ia);
        if constexpr (G == 2) off += variant_off<UB>(a, 1, jb);
        v[ia * NB + jb] = a.in[off];
      }
    double t[4 * NB];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      double col[NA], p[4];
#pragma unroll
      for (int ia = 0; ia < NA; ++ia) col[ia] = v[ia * NB + jb];
      cut_map<UA>(col, p);
#pragma unroll
      for (int sa = 0; sa < 4; ++sa) t[sa * NB + jb] = p[sa];
    }
    if constexpr (G == 1) {
#pragma unroll
      for (int sa = 0; sa < 4; ++sa) {
        const uint64_t o = ob + (uint64_t)sa * a.row_out[0];
        a.out[o] = t[sa];
        if (a.amax) amax_take(a, o, t[sa], mx);
      }
    } else {
#pragma unroll
      for (int sa = 0; sa < 4; ++sa) {
        double p[4];
        cut_map<UB>(t + sa * NB, p);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
          const uint64_t o = ob + (uint64_t)sa * a.row_out[0] + (uint64_t)sb * a.row_out[1];
          a.out[o] = p[sb];
          if (a.amax) amax_take(a, o, p[sb], mx);
        }
      }
    }
  }
  if (a.amax) amax_commit(a.amax, mx);
}

// several passes per launch (blockIdx.y selects the pass; one pass of each
// of several tensors): the variant is uniform over a workgroup
struct PassBatch {
  TransformPassArgs a[kPassBatch];
  uint32_t nblk[kPassBatch];  // workgroups of each pass (the first ones of its row)
  unsigned long long *zero;   // optional: cleared by the first workgroup
  int nzero;
};
__device__ inline void pass_dispatch(const TransformPassArgs &a, uint64_t bid, uint64_t nblk) {
  if (a.g == 1) {
    if (a.up[0]) pass_body<1, true, false>(a, bid, nblk);
    else pass_body<1, false, false>(a, bid, nblk);
  } else if (a.up[0]) {
    if (a.up[1]) pass_body<2, true, true>(a, bid, nblk);
    else pass_body<2, true, false>(a, bid, nblk);
  } else {
    if (a.up[1]) pass_body<2, false, true>(a, bid, nblk);
    else pass_body<2, false, false>(a, bid, nblk);
  }
}

__global__ void __launch_bounds__(256) transform_pass_kernel(PassBatch pb) {
  if (pb.zero && blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = (int)threadIdx.x; i < pb.nzero; i += (int)blockDim.x) pb.zero[i] = 0ull;
  const uint32_t nb = pb.nblk[blockIdx.y];
  if (blockIdx.x >= nb) return;  // whole workgroup
  pass_dispatch(pb.a[blockIdx.y], blockIdx.x, nb);
}

// The last pass level of some tensors and the per-entry transforms of others
// in one launch: blockIdx.y < np selects a pass, the rest a tensor, which
// runs on the first blocks[i] workgroups of its row (its own launch's grid).
struct TransformRows {
  uint32_t blocks[4];
};
__global__ void __launch_bounds__(256) transform_level_kernel(PassBatch pb, TransformBatch tb, TransformRows tr,
                                                              int np) {
  const int y = (int)blockIdx.y;
  if (y < np) {
    const uint32_t nb = pb.nblk[y];
    if (blockIdx.x < nb) pass_dispatch(pb.a[y], blockIdx.x, nb);
    return;
  }
  const uint32_t nb = tr.blocks[y - np];
  if (blockIdx.x >= nb) return;  // whole workgroup
  transform_range(tb.a[y - np], blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)nb * blockDim.x);
}

hipError_t launch_transform_level(const TransformPassArgs *pa, int np, const TransformArgs *ta, int nt,
                                  hipStream_t s) {
  if (np < 1 || np > kPassBatch || nt < 1 || nt > 4) return hipErrorInvalidValue;
  PassBatch pb{};
  TransformBatch tb{};
  TransformRows tr{};
  unsigned blocks = 1;
  for (int i = 0; i < np; ++i) {
    if (pa[i].nseg < 1 || pa[i].nseg > kPassSegs || pa[i].g < 1 || pa[i].g > 2) return hipErrorInvalidValue;
    pb.a[i] = pa[i];
    pb.nblk[i] = transform_grid(pa[i].nfree, pa[i].amax != nullptr);
    blocks = pb.nblk[i] > blocks ? pb.nblk[i] : blocks;
  }
  for (int i = 0; i < nt; ++i) {
    tb.a[i] = ta[i];
    tr.blocks[i] = transform_grid((1ull << (2 * ta[i].c)) << ta[i].o, ta[i].amax != nullptr);
    blocks = tr.blocks[i] > blocks ? tr.blocks[i] : blocks;
  }
  hipLaunchKernelGGL(transform_level_kernel, dim3(blocks, np + nt), dim3(256), 0, s, pb, tb, tr, np);
  return hipGetLastError();
}

hipError_t launch_transform_passes(const TransformPassArgs *args, int n, hipStream_t s, unsigned long long *zero,
                                   int nzero) {
  for (int i = 0; i < n; ++i)
    if (args[i].nseg < 1 || args[i].nseg > kPassSegs || args[i].g < 1 || args[i].g > 2)
      return hipErrorInvalidValue;
  for (int i0 = 0; i0 < n; i0 += kPassBatch) {
    PassBatch pb{};
    if (i0 == 0) {
      pb.zero = zero;
      pb.nzero = nzero;
    }
    const int cnt = n - i0 < kPassBatch ? n - i0 : kPassBatch;
    unsigned blocks = 1;
    for (int i = 0; i < cnt; ++i) {
      pb.a[i] = args[i0 + i];
      pb.nblk[i] = transform_grid(args[i0 + i].nfree, args[i0 + i].amax != nullptr);
      blocks = pb.nblk[i] > blocks ? pb.nblk[i] : blocks;
    }
    hipLaunchKernelGGL(transform_pass_kernel, dim3(blocks, cnt), dim3(256), 0, s, pb);
  }
  return hipGetLastError();
}

hipError_t launch_transform(const TransformArgs &a, hipStream_t s) {
  const uint64_t total = (1ull << (2 * a.c)) << a.o;
  hipLaunchKernelGGL(transform_kernel, dim3(transform_grid(total, a.amax != nullptr)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_transforms(const TransformArgs *args, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 4) {
    TransformBatch tb{};
    const int cnt = n - i0 < 4 ? n - i0 : 4;
    unsigned blocks = 1;
    for (int i = 0; i < cnt; ++i) {
      tb.a[i] = args[i0 + i];
      const uint64_t total = (1ull << (2 * args[i0 + i].c)) << args[i0 + i].o;
      const unsigned b = transform_grid(total, args[i0 + i].amax != nullptr);
      blocks = b > blocks ? b : blocks;
    }
    hipLaunchKernelGGL(transform_multi_kernel, dim3(blocks, cnt), dim3(256), 0, s, tb);
  }
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

hipError_t launch_absmax(const AbsMaxArgs *args, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += kPackBatch) {
    AbsMaxBatch ab{};
    const int cnt = n - i0 < kPackBatch ? n - i0 : kPackBatch;
    uint64_t most = 1;
    for (int i = 0; i < cnt; ++i) {
      ab.a[i] = args[i0 + i];
      const uint64_t total = 1ull << args[i0 + i].nbits;
      most = total > most ? total : most;
    }
    // about 8 entries per thread: fewer workgroups, fewer serialized atomics
    hipLaunchKernelGGL(absmax_kernel, dim3(grid_for(most / 8 + 1, kMaxGrid), cnt), dim3(256), 0, s, ab);
  }
  return hipGetLastError();
}

hipError_t launch_packs(const PackArgs *args, int n, hipStream_t s, const ScaleRec *sr) {
  for (int i0 = 0; i0 < n; i0 += kPackBatch) {
    PackBatch pb{};
    if (i0 == 0 && sr) pb.sr = *sr;
    const int cnt = n - i0 < kPackBatch ? n - i0 : kPackBatch;
    unsigned blocks = 1;
    for (int i = 0; i < cnt; ++i) {
      pb.a[i] = args[i0 + i];
      pb.nblk[i] = pack_blocks(args[i0 + i]);
      blocks = pb.nblk[i] > blocks ? pb.nblk[i] : blocks;
    }
    hipLaunchKernelGGL(pack_multi_kernel, dim3(blocks, cnt), dim3(256), 0, s, pb);
  }
  return hipGetLastError();
}

// ============================================= float16 split of final operands
// The final step of a float16-split plan reads each operand as two float16
// planes: with e the power of two that puts the operand's largest |value| in
// [2^14, 2^15) (float16 reaches 65504), hi = RNE16(v 2^e) and lo =
// RNE16(v 2^e - hi) (v 2^e - hi is exact in float32).  The output scale
// 2^-(ea + eb) times the plan's root scale is written for the epilogue.
// blockIdx.y selects the operand.
struct F16Split {
  const float *src[2];
  uint64_t n[2];
  uint16_t *hi[2], *lo[2];
  unsigned long long *maxbits;  // two entries, zero before the abs-max pass
  const double *root_scale;
  double *root_scale2;
};

// Operands whose length is a multiple of 4 and whose base is 16-byte aligned
// (the planner's layouts always are) are read and written four entries at a
// time; the scalar loop is the general case.
__device__ inline bool f16_vec_ok(const F16Split &a, int y) {
  return (a.n[y] & 3) == 0 && ((uintptr_t)a.src[y] & 15) == 0 && ((uintptr_t)a.hi[y] & 7) == 0 &&
         ((uintptr_t)a.lo[y] & 7) == 0;
}

__global__ void __launch_bounds__(256) f16_absmax_kernel(F16Split a) {
  __shared__ float red[256];
  const int y = blockIdx.y;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  float mx = 0.f;
  if (f16_vec_ok(a, y)) {
    const float4 *v = (const float4 *)a.src[y];
#pragma unroll 4
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.n[y] / 4; i += stride) {
      const float4 q = v[i];
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fmaxf(fabsf(q.z), fabsf(q.w))));
    }
  } else {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.n[y]; i += stride)
      mx = fmaxf(mx, fabsf(a.src[y][i]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(a.maxbits + y, (unsigned long long)__double_as_longlong((double)red[0]));
}

__device__ inline int f16_exponent(unsigned long long bits) {
  const double mx = __longlong_as_double((long long)bits);
  return mx > 0.0 ? 14 - ilogb(mx) : 0;
}

__global__ void __launch_bounds__(256) f16_split_kernel(F16Split a) {
  const int y = blockIdx.y;
  const int e = f16_exponent(a.maxbits[y]);
  if (blockIdx.x == 0 && y == 0 && threadIdx.x == 0)
    *a.root_scale2 = ldexp(*a.root_scale, -f16_exponent(a.maxbits[0]) - f16_exponent(a.maxbits[1]));
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (f16_vec_ok(a, y)) {
    const float4 *src = (const float4 *)a.src[y];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.n[y] / 4; i += stride) {
      const float4 q = src[i];
      const float v[4] = {ldexpf(q.x, e), ldexpf(q.y, e), ldexpf(q.z, e), ldexpf(q.w, e)};
      uint16_t hs[4], ls[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const _Float16 h = (_Float16)v[c];
        const _Float16 l = (_Float16)(v[c] - (float)h);
        hs[c] = __builtin_bit_cast(uint16_t, h);
        ls[c] = __builtin_bit_cast(uint16_t, l);
      }
      const uint2 hw = {(uint32_t)hs[0] | ((uint32_t)hs[1] << 16), (uint32_t)hs[2] | ((uint32_t)hs[3] << 16)};
      const uint2 lw = {(uint32_t)ls[0] | ((uint32_t)ls[1] << 16), (uint32_t)ls[2] | ((uint32_t)ls[3] << 16)};
      ((uint2 *)a.hi[y])[i] = hw;
      ((uint2 *)a.lo[y])[i] = lw;
    }
    return;
  }
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.n[y]; i += stride) {
    const float v = ldexpf(a.src[y][i], e);
    const _Float16 h = (_Float16)v;
    const _Float16 l = (_Float16)(v - (float)h);
    a.hi[y][i] = __builtin_bit_cast(uint16_t, h);
    a.lo[y][i] = __builtin_bit_cast(uint16_t, l);
  }
}

hipError_t launch_f16_split(const float *src0, uint64_t n0, uint16_t *hi0, uint16_t *lo0, const float *src1,
                            uint64_t n1, uint16_t *hi1, uint16_t *lo1, unsigned long long *maxbits,
                            const double *root_scale, double *root_scale2, hipStream_t s) {
  F16Split a{};
  a.src[0] = src0;
  a.src[1] = src1;
  a.n[0] = n0;
  a.n[1] = n1;
  a.hi[0] = hi0;
  a.hi[1] = hi1;
  a.lo[0] = lo0;
  a.lo[1] = lo1;
  a.maxbits = maxbits;
  a.root_scale = root_scale;
  a.root_scale2 = root_scale2;
  const uint64_t most = n0 > n1 ? n0 : n1;
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, s, maxbits, (uint64_t)2);
  hipLaunchKernelGGL(f16_absmax_kernel, dim3(grid_for(most / 4 + 1, kMaxGrid), 2), dim3(256), 0, s, a);
  hipLaunchKernelGGL(f16_split_kernel, dim3(grid_for(most / 4 + 1), 2), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ===================================================== heavy state selection
// Column L2 norms of a Pauli tensor [rows][cols] (Alg. 1: per output state,
// the norm over every edge permutation).  Pass 1: workgroup (x, y) sums the
// squares of 64 columns over row chunk y (4 row lanes, fixed-order lane
// sum); pass 2 adds the chunks in order and takes the square root.  The
// result is deterministic.
constexpr int kNormRows = 1024;  // rows per chunk
__global__ void __launch_bounds__(256) colnorm_partial_kernel(const double *T, uint64_t rows, uint64_t cols,
                                                              double *partial) {
  __shared__ double red[4][64];
  const uint64_t col = (uint64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int lane4 = threadIdx.x >> 6;
  const uint64_t r0 = (uint64_t)blockIdx.y * kNormRows;
  const uint64_t r1 = r0 + kNormRows < rows ? r0 + kNormRows : rows;
  double acc = 0.0;
  if (col < cols)
    for (uint64_t r = r0 + lane4; r < r1; r += 4) {
      const double v = T[r * cols + col];
      acc += v * v;
    }
  red[lane4][threadIdx.x & 63] = acc;
  __syncthreads();
  if (lane4 == 0 && col < cols)
    partial[(uint64_t)blockIdx.y * cols + col] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                                 red[3][threadIdx.x];
}

__global__ void __launch_bounds__(256) colnorm_final_kernel(const double *partial, uint64_t chunks, uint64_t cols,
                                                            double *norms) {
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < cols; c += (uint64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (uint64_t k = 0; k < chunks; ++k) s += partial[k * cols + c];
    norms[c] = sqrt(s);
  }
}

uint64_t colnorm_scratch_entries(uint64_t rows, uint64_t cols) {
  return ((rows + kNormRows - 1) / kNormRows) * cols;
}

hipError_t launch_column_norms(const double *T, uint64_t rows, uint64_t cols, double *partial, double *norms,
                               hipStream_t s) {
  const uint64_t chunks = (rows + kNormRows - 1) / kNormRows;
  if (chunks > 65535 || cols == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(colnorm_partial_kernel, dim3((unsigned)((cols + 63) / 64), (unsigned)chunks), dim3(256), 0, s,
                     T, rows, cols, partial);
  hipLaunchKernelGGL(colnorm_final_kernel, dim3(grid_for(cols)), dim3(256), 0, s, partial, chunks, cols, norms);
  return hipGetLastError();
}

// dst[r][y] = src[r][states[y]] for y < count, 0 for the padding columns
// y in [count, dst_cols)
__global__ void __launch_bounds__(256) gather_columns_kernel(const double *src, uint64_t rows, uint64_t src_cols,
                                                             const int32_t *states, uint64_t count,
                                                             uint64_t dst_cols, double *dst) {
  const uint64_t total = rows * dst_cols;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = e / dst_cols, y = e - r * dst_cols;
    dst[e] = y < count ? src[r * src_cols + (uint64_t)states[y]] : 0.0;
  }
}

hipError_t launch_gather_columns(const double *src, uint64_t rows, uint64_t src_cols, const int32_t *states,
                                 uint64_t count, uint64_t dst_cols, double *dst, hipStream_t s) {
  if (count > dst_cols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_columns_kernel, dim3(grid_for(rows * dst_cols)), dim3(256), 0, s, src, rows, src_cols,
                     states, count, dst_cols, dst);
  return hipGetLastError();
}

// one thread stores the device's constant-rate clock (a timestamp that
// orders work across streams of one device)
__global__ void stamp_kernel(unsigned long long *dst) {
  if (threadIdx.x == 0) dst[0] = wall_clock64();
}

hipError_t launch_stamp(unsigned long long *dst, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, dst);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *buf, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(grid_for(n)), dim3(256), 0, s, buf, n);
  return hipGetLastError();
}

// Largest |a - ref| and largest |ref| over two vectors (a float32 or
// float64, ref float64), as the bit patterns of non-negative doubles in
// out[0] and out[1] (cleared by the caller).  The planner's error check of a
// candidate plan against a float64 reference result.
__global__ void __launch_bounds__(256) max_abs_diff_kernel(const void *a, int a_f32, const double *ref, uint64_t n,
                                                           unsigned long long *out) {
  __shared__ double rd[256], rr[256];
  double d = 0.0, r = 0.0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const double x = a_f32 ? (double)((const float *)a)[i] : ((const double *)a)[i];
    const double y = ref[i];
    d = fmax(d, fabs(x - y));
    r = fmax(r, fabs(y));
  }
  rd[threadIdx.x] = d;
  rr[threadIdx.x] = r;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + w]);
      rr[threadIdx.x] = fmax(rr[threadIdx.x], rr[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(rd[0]));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(rr[0]));
  }
}

hipError_t launch_max_abs_diff(const void *a, int a_f32, const double *ref, uint64_t n, unsigned long long *out,
                               hipStream_t s) {
  hipLaunchKernelGGL(max_abs_diff_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, s, a, a_f32, ref, n, out);
  return hipGetLastError();
}

hipError_t launch_scale_f64(double *buf, uint64_t n, double sc, hipStream_t s) {
  hipLaunchKernelGGL(scale_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, buf, n, sc);
  return hipGetLastError();
}

static int device_cus() {
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

// Split count (log2) of a step: only when its tiles cannot fill the device
// and k is long; every split keeps at least 256 k, the splits of all tiles
// give about two workgroups per CU, and the partial buffer bounds the count.
// Steps that write tile statistics are never split.
static int splitk_log2(const GemmArgs &g, uint64_t tiles, uint64_t mn) {
  if (!g.partial || g.tkey || g.kpad < 9) return 0;
  const uint64_t cus = (uint64_t)device_cus();
  if (cus == 0 || tiles >= cus) return 0;
  int ks = 0;
  while ((tiles << ks) < 2 * cus && ks < g.kpad - 8) ++ks;
  while (ks > 0 && (mn << ks) * 8 > g.partial_bytes) --ks;
  return ks;
}

template <int P, int BM, int BN, int BK>
static hipError_t launch_gemm_t(GemmArgs g, hipStream_t s, bool general) {
  using S = GemmShape<P, BM, BN, BK>;
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  const uint64_t tilesM = (M + BM - 1) / BM, tilesN = (N + BN - 1) / BN;
  const uint64_t tiles = tilesM * tilesN;
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  // long k on whole 128 x 128 tiles that fill the device: the deep-ring kernel
  if (!general && BM == 128 && BN == 128 && gemm_long_eligible(P, g, (uint64_t)device_cus()))
    return launch_gemm_long(P, g, s);
  prepare_gemm_args(g, P, BM, BN);
  static_assert(S::LDS_BYTES <= 81920, "two workgroups per CU need at most 80 KiB of LDS each");
  g.ksplit = splitk_log2(g, tiles, M * N);
  const uint64_t grid = tiles << g.ksplit;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  if (P != 0 && g.kpad - g.ksplit > 8)
    hipLaunchKernelGGL((gemm_kernel<P, BM, BN, BK, true>), dim3((unsigned)grid), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_kernel<P, BM, BN, BK, false>), dim3((unsigned)grid), dim3(256), 0, s, g);
  if (g.ksplit) hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(M * N)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// tile ids: 0 = 128x128, 1 = 64x64, 2 = 32x32
template <int P, int BK>
static hipError_t launch_gemm_bk(const GemmArgs &g, int tile, hipStream_t s, bool general) {
  switch (tile) {
    case 0: return launch_gemm_t<P, 128, 128, BK>(g, s, general);
    case 1: return launch_gemm_t<P, 64, 64, BK>(g, s, general);
    default: return launch_gemm_t<P, 32, 32, BK>(g, s, general);
  }
}

hipError_t launch_gemm(int prec, const GemmArgs &g, int tile, hipStream_t s, bool general) {
  const int kp = g.kpad;
  switch (prec) {
    case 0: return launch_gemm_bk<0, 16>(g, tile, s, general);
    case 1: return kp >= 5 ? launch_gemm_bk<1, 32>(g, tile, s, general) : launch_gemm_bk<1, 16>(g, tile, s, general);
    case 2: return launch_gemm_bk<2, 32>(g, tile, s, general);
    case 3: return launch_gemm_bk<3, 32>(g, tile, s, general);
    default: return launch_gemm_bk<4, 32>(g, tile, s, general);
  }
}

// =========================================================== grouped launches
// One launch runs the same kind of work of many reconstructions.  Record r
// owns workgroups [first[r], first[r + 1]) of the grid and runs them as the
// workgroups 0.. of its own single-record launch would, so every entry
// sees the same arithmetic as in that launch.
__device__ inline int group_record(const uint32_t *first, int n, uint32_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) grouped_pass_kernel(const TransformPassArgs *recs, const uint32_t *first,
                                                           int n) {
  const int r = group_record(first, n, blockIdx.x);
  pass_dispatch(recs[r], blockIdx.x - first[r], first[r + 1] - first[r]);
}

__global__ void __launch_bounds__(256) grouped_transform_kernel(const TransformArgs *recs, const uint32_t *first,
                                                                int n) {
  const int r = group_record(first, n, blockIdx.x);
  const uint64_t nb = first[r + 1] - first[r];
  transform_range(recs[r], (blockIdx.x - first[r]) * (uint64_t)blockDim.x + threadIdx.x, nb * blockDim.x);
}

__global__ void __launch_bounds__(256) grouped_zero_kernel(const ZeroRec *recs, int n) {
  const ZeroRec &z = recs[blockIdx.x];
  for (uint64_t i = threadIdx.x; i < z.n; i += blockDim.x) z.p[i] = 0ull;
}

__global__ void __launch_bounds__(256) grouped_absmax_kernel(const AbsMaxArgs *recs, const uint32_t *first, int n) {
  const int r = group_record(first, n, blockIdx.x);
  const AbsMaxArgs &a = recs[r];
  __shared__ double red[256];
  const uint64_t total = 1ull << a.nbits;
  const uint64_t nb = first[r + 1] - first[r];
  double mx = 0.0;
  for (uint64_t e = (blockIdx.x - first[r]) * (uint64_t)blockDim.x + threadIdx.x; e < total; e += nb * blockDim.x)
    mx = fmax(mx, gathered_abs(a, e));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(a.out, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void __launch_bounds__(64) grouped_scale_kernel(const ScaleRec *recs, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  write_scales(recs[r]);
}

__global__ void __launch_bounds__(256) grouped_pack_kernel(const PackArgs *recs, const uint32_t *first, int n) {
  __shared__ double tile[kPackTileEntries + 32];
  const int r = group_record(first, n, blockIdx.x);
  pack_range(recs[r], blockIdx.x - first[r], first[r + 1] - first[r], tile);
}

template <int P, int BM, int BN, int BK, bool A64>
__global__ void __launch_bounds__(256) grouped_gemm_kernel(const GemmArgs *recs, const uint32_t *first, int n) {
  __shared__ __attribute__((aligned(16))) char smem[GemmShape<P, BM, BN, BK>::LDS_BYTES];
  const int r = group_record(first, n, blockIdx.x);
  gemm_tile<P, BM, BN, BK, A64>(recs[r], blockIdx.x - first[r], smem);
}

uint32_t grouped_pass_blocks(const TransformPassArgs &a) { return transform_grid(a.nfree, a.amax != nullptr); }
uint32_t grouped_transform_blocks(const TransformArgs &a) {
  return transform_grid((1ull << (2 * a.c)) << a.o, a.amax != nullptr);
}
uint32_t grouped_absmax_blocks(const AbsMaxArgs &a) { return grid_for((1ull << a.nbits) / 8 + 1, kMaxGrid); }
uint32_t grouped_pack_blocks(const PackArgs &a) { return pack_blocks(a); }

hipError_t launch_grouped_passes(const TransformPassArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                 hipStream_t s) {
  if (n < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_pass_kernel, dim3(blocks), dim3(256), 0, s, recs, first, n);
  return hipGetLastError();
}
hipError_t launch_grouped_transforms(const TransformArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                     hipStream_t s) {
  if (n < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_transform_kernel, dim3(blocks), dim3(256), 0, s, recs, first, n);
  return hipGetLastError();
}
hipError_t launch_grouped_zero(const ZeroRec *recs, int n, hipStream_t s) {
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_zero_kernel, dim3(n), dim3(256), 0, s, recs, n);
  return hipGetLastError();
}
hipError_t launch_grouped_absmax(const AbsMaxArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                 hipStream_t s) {
  if (n < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_absmax_kernel, dim3(blocks), dim3(256), 0, s, recs, first, n);
  return hipGetLastError();
}
hipError_t launch_grouped_scales(const ScaleRec *recs, int n, hipStream_t s) {
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_scale_kernel, dim3((n + 63) / 64), dim3(64), 0, s, recs, n);
  return hipGetLastError();
}
hipError_t launch_grouped_packs(const PackArgs *recs, const uint32_t *first, int n, uint32_t blocks, hipStream_t s) {
  if (n < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grouped_pack_kernel, dim3(blocks), dim3(256), 0, s, recs, first, n);
  return hipGetLastError();
}

GemmClass gemm_class(int prec, const GemmArgs &g, int tile) {
  GemmClass c{};
  c.prec = prec;
  c.tile = tile;
  c.bk = prec == 0 ? 16 : (prec == 1 ? (g.kpad >= 5 ? 32 : 16) : 32);
  const int bm = tile == 0 ? 128 : (tile == 1 ? 64 : 32);
  const uint64_t tiles = (((1ull << g.lm) + bm - 1) / bm) * (((1ull << g.ln) + bm - 1) / bm);
  c.ksplit = splitk_log2(g, tiles, 1ull << (g.lm + g.ln));
  c.a64 = prec != 0 && g.kpad - c.ksplit > 8;
  c.tiles = tiles;
  return c;
}

template <int P, int BM, int BK>
static void launch_gg(bool a64, const GemmArgs *recs, const uint32_t *first, int n, uint32_t blocks, hipStream_t s) {
  if constexpr (P == 0) {
    hipLaunchKernelGGL((grouped_gemm_kernel<P, BM, BM, BK, false>), dim3(blocks), dim3(256), 0, s, recs, first, n);
  } else {
    if (a64)
      hipLaunchKernelGGL((grouped_gemm_kernel<P, BM, BM, BK, true>), dim3(blocks), dim3(256), 0, s, recs, first, n);
    else
      hipLaunchKernelGGL((grouped_gemm_kernel<P, BM, BM, BK, false>), dim3(blocks), dim3(256), 0, s, recs, first, n);
  }
}

template <int P, int BK>
static void launch_gg_tile(int tile, bool a64, const GemmArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                           hipStream_t s) {
  switch (tile) {
    case 0: launch_gg<P, 128, BK>(a64, recs, first, n, blocks, s); break;
    case 1: launch_gg<P, 64, BK>(a64, recs, first, n, blocks, s); break;
    default: launch_gg<P, 32, BK>(a64, recs, first, n, blocks, s); break;
  }
}

hipError_t launch_grouped_gemm(const GemmClass &c, const GemmArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                               hipStream_t s) {
  if (n < 1 || blocks < 1 || c.ksplit != 0 || c.tile < 0 || c.tile > 2) return hipErrorInvalidValue;
  switch (c.prec) {
    case 0: launch_gg_tile<0, 16>(c.tile, false, recs, first, n, blocks, s); break;
    case 1:
      if (c.bk == 32) launch_gg_tile<1, 32>(c.tile, c.a64, recs, first, n, blocks, s);
      else launch_gg_tile<1, 16>(c.tile, c.a64, recs, first, n, blocks, s);
      break;
    case 2: launch_gg_tile<2, 32>(c.tile, c.a64, recs, first, n, blocks, s); break;
    case 3: launch_gg_tile<3, 32>(c.tile, c.a64, recs, first, n, blocks, s); break;
    default: launch_gg_tile<4, 32>(c.tile, c.a64, recs, first, n, blocks, s); break;
  }
  return hipGetLastError();
}

}  // namespace tqc
