// Many independent reconstructions in one persistent launch.
//
// Three short launches over all jobs come first: the Pauli transform of
// every raw tensor, the largest |value| of every leaf operand and the
// power-of-two exponents per job (the same operand rescaling as a single
// reconstruction, so results agree bit for bit).  Then every job's work is
// cut into items: chunks of operand packing and GEMM tiles of each pairwise
// step.  Items are listed in topological level order across all jobs (packs,
// then steps by depth in the contraction tree) and claimed in that order from
// one global counter, so an item only ever waits for items claimed before it
// by workgroups that are already running: the grid drains whatever its size.
// A unit (one transform, pack or step) counts its finished items; a waiting
// item spins on its producers' counters with agent-scope acquire loads,
// bounded by a spin limit (on overrun it sets an error flag and skips its
// work, so every wave still reaches the exit).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.hpp"
#include "dev_ops.hpp"

namespace tqc {

constexpr uint64_t kChunkElems = 4096;

__device__ inline unsigned int load_acquire(const unsigned int *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int P>
struct BatchLds {
  static constexpr int a = GemmShape<P, 128, 128, 32>::LDS_BYTES;
  static constexpr int b = GemmShape<P, 128, 128, 16>::LDS_BYTES;
  static constexpr int bytes = a > b ? a : b;
};

template <int P, int BM, int BN>
__device__ inline void gemm_tile_k(const GemmArgs &g, uint64_t t, char *smem) {
  if constexpr (P == 0) {
    gemm_tile<P, BM, BN, 16>(g, t, smem);
  } else if constexpr (P == 1) {
    if (g.lk > 8) gemm_tile<P, BM, BN, 32, true>(g, t, smem);
    else if (g.kpad >= 5) gemm_tile<P, BM, BN, 32>(g, t, smem);
    else gemm_tile<P, BM, BN, 16>(g, t, smem);
  } else {
    if (g.lk > 8) gemm_tile<P, BM, BN, 32, true>(g, t, smem);
    else gemm_tile<P, BM, BN, 32>(g, t, smem);
  }
}

template <int P>
__global__ void __launch_bounds__(256) batch_kernel(BatchDesc d) {
  __shared__ __attribute__((aligned(16))) char smem[BatchLds<P>::bytes];
  // The claim / dispatch scalars live at the head of the tile scratch: every
  // thread copies them to registers before the first barrier of the item's
  // work, and thread 0 rewrites them only after the item's last barrier.
  unsigned long long &s_item = *(unsigned long long *)smem;
  int &s_unit = *(int *)(smem + 8);
  int &s_ok = *(int *)(smem + 12);
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_item = d.first_item + atomicAdd(d.next, 1ull);
    __syncthreads();
    const unsigned long long item = s_item;
    if (item >= d.total) break;
    if (tid == 0) {
      int lo = 0, hi = d.nunits - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.units[mid].first <= item) lo = mid;
        else hi = mid - 1;
      }
      s_unit = lo;
      int ok = 1;
      const int deps[2] = {d.units[lo].dep0, d.units[lo].dep1};
      for (int k = 0; k < 2 && ok && !d.nowait; ++k) {
        const int dep = deps[k];
        if (dep < 0) continue;
        const unsigned int need = (unsigned int)d.units[dep].ntiles;
        unsigned long long spins = 0;
        while (load_acquire(&d.counters[dep]) < need) {
          if (++spins > d.spin_limit) {
            atomicOr(d.error, 1u);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      atomicMin(&d.job_start[d.units[lo].job], (unsigned long long)wall_clock64());
      s_ok = ok;
    }
    __syncthreads();
    const int unit = s_unit;
    const int ok = s_ok;
    const BatchUnit &u = d.units[unit];
    const uint64_t t = item - u.first;
    if (ok) {
      if (u.kind == UNIT_PACK) {
        const PackArgs &a = d.pargs[u.arg];
        const uint64_t total = 1ull << a.nbits;
        const uint64_t e1 = (t + 1) * kChunkElems < total ? (t + 1) * kChunkElems : total;
        for (uint64_t e = t * kChunkElems + tid; e < e1; e += 256) pack_elem(a, e);
      } else {
        const GemmArgs &g = d.gargs[u.arg];
        switch (u.tile) {
          case 0: gemm_tile_k<P, 128, 128>(g, t, smem); break;
          case 1: gemm_tile_k<P, 64, 64>(g, t, smem); break;
          default: gemm_tile_k<P, 32, 32>(g, t, smem); break;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      __threadfence();  // release this item's results at agent scope
      const unsigned int old = atomicAdd(&d.counters[unit], 1u);
      if (u.is_root && old + 1 == (unsigned int)u.ntiles)
        atomicMax(&d.job_end[u.job], (unsigned long long)wall_clock64());
    }
  }
}

__global__ void batch_reset_kernel(BatchDesc d, int njobs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= d.nlevels) d.next[i] = 0;  // one claim counter per launch
  if (i == 0) *d.error = 0;
  for (int u = i; u < d.nunits; u += gridDim.x * blockDim.x) d.counters[u] = 0;
  for (int j = i; j < njobs; j += gridDim.x * blockDim.x) {
    d.job_start[j] = ~0ull;
    d.job_end[j] = 0;
  }
  for (int l = i; l < d.nleaves; l += gridDim.x * blockDim.x) d.maxbits[l] = 0;
}

// pre-pass kernels: blockIdx.y selects the tensor / leaf / job
__global__ void __launch_bounds__(256) batch_transform_kernel(const TransformArgs *targs) {
  const TransformArgs &a = targs[blockIdx.y];
  const uint64_t total = (1ull << (2 * a.c)) << a.o;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    transform_elem(a, e);
}

__global__ void __launch_bounds__(256) batch_absmax_kernel(const AbsMaxArgs *aargs) {
  __shared__ double red[256];
  const AbsMaxArgs &a = aargs[blockIdx.y];
  const uint64_t total = 1ull << a.nbits;
  double mx = 0.0;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    mx = fmax(mx, gathered_abs(a, e));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(a.out, (unsigned long long)__double_as_longlong(red[0]));
}

// same exponent rule as the single-plan path: e = -floor(log2 max), output
// scale 2^(-K - sum e)
__global__ void batch_scale_kernel(BatchDesc d, int njobs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  int sum = 0;
  for (int l = d.job_leaf0[j]; l < d.job_leaf0[j + 1]; ++l) {
    const double mx = __longlong_as_double((long long)d.maxbits[l]);
    const int e = mx > 0.0 ? -ilogb(mx) : 0;
    d.exps[l] = e;
    sum += e;
  }
  d.root_scale[j] = ldexp(1.0, -d.job_cuts[j] - sum);
}

static unsigned pre_grid(uint64_t elems) {
  uint64_t b = (elems + 255) / 256;
  if (b > 1024) b = 1024;
  return (unsigned)(b ? b : 1);
}

static void launch_persistent(int prec, const BatchDesc &d, int grid, hipStream_t s) {
  switch (prec) {
    case 0: hipLaunchKernelGGL(batch_kernel<0>, dim3(grid), dim3(256), 0, s, d); break;
    case 1: hipLaunchKernelGGL(batch_kernel<1>, dim3(grid), dim3(256), 0, s, d); break;
    case 2: hipLaunchKernelGGL(batch_kernel<2>, dim3(grid), dim3(256), 0, s, d); break;
    default: hipLaunchKernelGGL(batch_kernel<3>, dim3(grid), dim3(256), 0, s, d); break;
  }
}

hipError_t launch_batch(int prec, const BatchDesc &d, int njobs, int grid, int by_level,
                        hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(64), dim3(256), 0, s, d, njobs);
  if (d.ntransforms > 0)
    hipLaunchKernelGGL(batch_transform_kernel, dim3(pre_grid(d.max_transform_elems), d.ntransforms),
                       dim3(256), 0, s, d.targs);
  if (d.nleaves > 0) {
    hipLaunchKernelGGL(batch_absmax_kernel, dim3(pre_grid(d.max_leaf_elems), d.nleaves), dim3(256), 0, s,
                       d.aargs);
    hipLaunchKernelGGL(batch_scale_kernel, dim3((njobs + 255) / 256), dim3(256), 0, s, d, njobs);
  }
  if (!by_level) {
    BatchDesc e = d;
    e.nowait = 0;
    e.first_item = 0;
    e.total = d.level_first[d.nlevels];
    launch_persistent(prec, e, grid, s);
  } else {
    // one launch per level of the contraction trees: the launch boundary
    // orders the levels, so no item waits for another
    for (int L = 0; L < d.nlevels; ++L) {
      BatchDesc e = d;
      e.nowait = 1;
      e.first_item = d.level_first[L];
      e.total = d.level_first[L + 1];
      e.next = d.next + 1 + L;
      if (e.total > e.first_item) launch_persistent(prec, e, grid, s);
    }
  }
  return hipGetLastError();
}

int batch_blocks_per_cu(int prec) {
  int nb = 0;
  hipError_t e = hipSuccess;
  switch (prec) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<0>, 256, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<1>, 256, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<2>, 256, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<3>, 256, 0); break;
  }
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace tqc
