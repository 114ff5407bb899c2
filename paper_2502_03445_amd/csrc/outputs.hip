// Output forms of a reconstructed probability vector: top-k (the sum of the
// top |HSS| entries is P_HSS^max, Eq. (10)) and marginals / the total
// probability.  Both are HBM-bound scans; both are deterministic (integer
// atomics only, float64 sums in a fixed order).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_ops.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace tqc {

// ================================================================ top-k
// Exact selection of the k-th largest value by radix select over an
// order-preserving integer key (11-bit digits, most significant first), then
// collection of every entry above that value plus the lowest-index entries
// equal to it, then a bitonic sort of the k winners by (value desc, index
// asc).  The fast forms gather a candidate superset (up to kMaxK entries)
// and place the first k by rank instead: each candidate's position in the
// order (value desc, index asc) is the number of candidates that sort before
// it, counted in parallel over 256 x 256 blocks of candidate pairs.

constexpr int kDigitBits = 11;
constexpr int kBins = 1 << kDigitBits;
constexpr uint64_t kChunk = 1ull << 16;  // elements per block in ordered passes
constexpr uint64_t kChunkGrid = 2048;     // largest grid of the exact passes (grid-strided)
constexpr int kMaxK = 4096;

struct TopkState {
  unsigned long long prefix;  // resolved high key bits
  int hi_shift;               // bits >= hi_shift are resolved
  int pad;
  unsigned long long kr;      // entries still needed among those matching prefix
  unsigned long long n_gt;    // slots used by entries strictly above the threshold
  unsigned long long ncand;   // fast path: candidates >= the chunk-max threshold
  unsigned int fallback;      // fast path could not decide: run the exact passes
  unsigned int pad2;
  unsigned long long nq;      // tile form: tiles whose maximum reaches the threshold
};

// keys of an already-keyed array (dtype 2)
__device__ inline uint64_t sort_key_any(const void *p, int dtype, uint64_t i);

__device__ inline uint64_t sort_key(const void *p, int dtype, uint64_t i) {
  if (dtype == 1) {
    uint32_t u = ((const uint32_t *)p)[i];
    return (u & 0x80000000u) ? (uint64_t)(~u) : (uint64_t)(u | 0x80000000u);
  }
  uint64_t u = ((const uint64_t *)p)[i];
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline uint64_t sort_key_any(const void *p, int dtype, uint64_t i) {
  return dtype == 2 ? ((const uint64_t *)p)[i] : sort_key(p, dtype, i);
}

__device__ inline double key_value(uint64_t key, int dtype) {
  if (dtype == 1) {
    uint32_t k = (uint32_t)key;
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return (double)__builtin_bit_cast(float, u);
  }
  uint64_t u = (key & 0x8000000000000000ull) ? (key & 0x7fffffffffffffffull) : ~key;
  return __builtin_bit_cast(double, u);
}

__device__ inline bool gated_off(const unsigned int *gate) { return gate && *gate == 0; }

// Appends the flagged entries of a wave to the candidate list with one
// atomic per wave (slot order inside a wave by lane); every lane of the wave
// must call it.  The count keeps growing past kMaxK so that an overflow is
// seen by the sort, which then raises the fallback flag.
__device__ inline void append_candidate(bool hit, uint64_t key, uint64_t idx, TopkState *fast, uint64_t *cand_key,
                                        uint64_t *cand_idx) {
  const unsigned long long bal = __ballot(hit);
  if (!bal) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)bal) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(&fast->ncand, (unsigned long long)__popcll(bal));
  base = __shfl(base, leader, 64);
  if (hit) {
    const unsigned long long slot = base + __popcll(bal & ((1ull << lane) - 1ull));
    if (slot < (unsigned long long)kMaxK) {
      cand_key[slot] = key;
      cand_idx[slot] = idx;
    }
  }
}

__global__ void __launch_bounds__(256) topk_init(TopkState *st, unsigned long long *hist,
                                                 int keybits, int k, const unsigned int *gate) {
  if (gated_off(gate)) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->prefix = 0;
    st->hi_shift = keybits;
    st->kr = (unsigned long long)k;
    st->n_gt = 0;
  }
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
}

__global__ void __launch_bounds__(256) topk_hist(const void *p, int dtype, uint64_t len,
                                                 const TopkState *st, unsigned long long *hist,
                                                 int bits, const unsigned int *gate) {
  if (gated_off(gate)) return;
  __shared__ unsigned int lh[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const int hs = st->hi_shift;
  const uint64_t prefix = st->prefix;
  const int shift = hs - bits;
  const uint64_t mask = (1ull << bits) - 1;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t key = sort_key_any(p, dtype, i);
    const bool match = (hs >= 64) ? true : ((key >> hs) == (prefix >> hs));
    // lanes with the same bin are counted by one atomic (fewer LDS conflicts)
    unsigned long long pending = __ballot(match);
    const unsigned int bin = (unsigned int)((key >> shift) & mask);
    const int lane = threadIdx.x & 63;
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const unsigned int lb = __shfl(bin, leader, 64);
      const unsigned long long same = __ballot(match && bin == lb) & pending;
      if (lane == leader) atomicAdd(&lh[lb], (unsigned int)__popcll(same));
      pending &= ~same;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], (unsigned long long)lh[b]);
}

// Walks the bins from the top: thread t owns the t-th group of `per`
// consecutive bins (from the largest down); group totals are prefix-summed
// and the one thread whose group holds the kr-th entry resolves the digit.
__global__ void __launch_bounds__(256) topk_select(TopkState *st, unsigned long long *hist, int bits,
                                                   const unsigned int *gate) {
  if (gated_off(gate)) return;
  __shared__ unsigned long long grp[4];  // per-wave totals
  const int nb = 1 << bits;
  const int per = (nb + 255) / 256;
  const int t = threadIdx.x;
  const int shift = st->hi_shift - bits;
  const unsigned long long kr = st->kr;
  unsigned long long mine = 0;
  for (int j = 0; j < per; ++j) {
    const int r = t * per + j;  // rank from the top
    if (r < nb) mine += hist[nb - 1 - r];
  }
  // exclusive prefix of the 256 group totals: within each wave by shuffles,
  // then the totals of the waves below
  const int lane = t & 63, wave = t >> 6;
  unsigned long long incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, (unsigned int)o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) grp[wave] = incl;
  __syncthreads();
  unsigned long long before = incl - mine;
  for (int w = 0; w < wave; ++w) before += grp[w];
  if (before < kr && before + mine >= kr) {
    unsigned long long cum = before;
    for (int j = 0; j < per; ++j) {
      const int r = t * per + j;
      if (r >= nb) break;
      const int b = nb - 1 - r;
      const unsigned long long h = hist[b];
      if (cum + h >= kr) {
        st->prefix |= (unsigned long long)b << shift;
        st->kr = kr - cum;
        break;
      }
      cum += h;
    }
  }
  __syncthreads();
  if (t == 0) st->hi_shift = shift;
  for (int b = t; b < kBins; b += blockDim.x) hist[b] = 0;
}

// entries strictly above the threshold go to candidate slots [0, n_gt);
// per-block counts of entries equal to it feed the ordered pass
__global__ void __launch_bounds__(256) topk_collect_gt(const void *p, int dtype, uint64_t len,
                                                       TopkState *st, uint64_t *cand_key,
                                                       uint64_t *cand_idx,
                                                       unsigned long long *blockcnt,
                                                       const unsigned int *gate) {
  if (gated_off(gate)) return;
  __shared__ unsigned int cnt;
  const uint64_t tau = st->prefix;
  const uint64_t nchunks = (len + kChunk - 1) / kChunk;
  // chunks grid-strided (a small grid costs little when the gate is off)
  for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const uint64_t lo = c * kChunk;
    const uint64_t hi = lo + kChunk < len ? lo + kChunk : len;
    unsigned int mine = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const uint64_t key = sort_key(p, dtype, i);
      if (key > tau) {
        const unsigned long long s = atomicAdd(&st->n_gt, 1ull);
        cand_key[s] = key;
        cand_idx[s] = i;
      } else if (key == tau) {
        ++mine;
      }
    }
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) blockcnt[c] = cnt;
  }
}

// exclusive scan of the per-block equal counts (one block, fixed order)
__global__ void __launch_bounds__(1024) topk_scan(unsigned long long *blockcnt, uint64_t nblocks,
                                                  const unsigned int *gate) {
  if (gated_off(gate)) return;
  __shared__ unsigned long long part[1024];
  const uint64_t per = (nblocks + 1023) / 1024;
  const uint64_t b0 = threadIdx.x * per;
  unsigned long long s = 0;
  for (uint64_t b = b0; b < b0 + per && b < nblocks; ++b) s += blockcnt[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int t = 0; t < 1024; ++t) {
      const unsigned long long v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (uint64_t b = b0; b < b0 + per && b < nblocks; ++b) {
    const unsigned long long v = blockcnt[b];
    blockcnt[b] = run;
    run += v;
  }
}

// equal entries in index order: the first kr of them are selected
__global__ void __launch_bounds__(256) topk_collect_eq(const void *p, int dtype, uint64_t len,
                                                       const TopkState *st, int k,
                                                       uint64_t *cand_key, uint64_t *cand_idx,
                                                       const unsigned long long *blockpre,
                                                       const unsigned int *gate) {
  if (gated_off(gate)) return;
  const unsigned long long need = st->kr;
  const uint64_t tau = st->prefix;
  const uint64_t nchunks = (len + kChunk - 1) / kChunk;
  const unsigned long long slot0 = (unsigned long long)k - need;
  __shared__ unsigned int wcount[4];
  __shared__ unsigned long long run;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // chunks grid-strided (a small grid costs little when the gate is off)
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const unsigned long long base = blockpre[ch];
    if (base >= need) continue;  // uniform over the block
    const uint64_t lo = ch * kChunk;
    const uint64_t hi = lo + kChunk < len ? lo + kChunk : len;
    if (threadIdx.x == 0) run = base;
    __syncthreads();
    for (uint64_t c = lo; c < hi; c += blockDim.x) {
      const uint64_t i = c + threadIdx.x;
      const bool eq = (i < hi) && (sort_key(p, dtype, i) == tau);
      const unsigned long long bal = __ballot(eq);
      const unsigned int below = __popcll(bal & ((1ull << lane) - 1ull));
      if (lane == 0) wcount[wave] = __popcll(bal);
      __syncthreads();
      unsigned long long r = run;
      for (int w = 0; w < wave; ++w) r += wcount[w];
      r += below;
      if (eq && r < need) {
        cand_key[slot0 + r] = tau;
        cand_idx[slot0 + r] = i;
      }
      __syncthreads();
      if (threadIdx.x == 0) run += wcount[0] + wcount[1] + wcount[2] + wcount[3];
      __syncthreads();
      if (run >= need) break;
    }
    __syncthreads();
  }
}

// bitonic sort of the k selected entries (padded to a power of two) by
// (key desc, index asc)
__global__ void __launch_bounds__(1024) topk_sort(const uint64_t *cand_key, const uint64_t *cand_idx,
                                                  int k, int dtype, uint64_t *idx_out,
                                                  double *val_out, const unsigned int *gate) {
  if (gated_off(gate)) return;
  // keys and indices, 2 x n entries (dynamic: 16 n bytes, n = k rounded up
  // to a power of two), so that the launch of a small k fits on a CU beside
  // another reconstruction's running final step
  extern __shared__ uint64_t sort_lds[];
  const int cnt = k;
  int n = 1;
  while (n < cnt) n <<= 1;
  uint64_t *sk = sort_lds, *si = sort_lds + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (i < cnt) {
      sk[i] = cand_key[i];
      si[i] = cand_idx[i];
    } else {
      sk[i] = 0;
      si[i] = ~0ull;
    }
  }
  __syncthreads();
  // "before(a, b)": a sorts earlier than b
  auto before = [](uint64_t ka, uint64_t ia, uint64_t kb, uint64_t ib) {
    return ka > kb || (ka == kb && ia < ib);
  };
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool asc = ((lo & size) == 0);
        const bool swap = asc ? before(sk[hi], si[hi], sk[lo], si[lo])
                              : before(sk[lo], si[lo], sk[hi], si[hi]);
        if (swap) {
          uint64_t a = sk[lo]; sk[lo] = sk[hi]; sk[hi] = a;
          a = si[lo]; si[lo] = si[hi]; si[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    idx_out[i] = si[i];
    val_out[i] = key_value(sk[i], dtype);
  }
}

// Candidate ranks.  The count of candidates is fast->ncand; outside
// [k, kMaxK] the fast form cannot decide and the placement raises the
// fallback flag.  Keys and indices are distinct pairs (every output index is
// a candidate at most once), so the ranks are a permutation of [0, count).
// partial[bj * kMaxK + i] = how many of candidates [256 bj, 256 bj + 256)
// sort before candidate i.
constexpr int kRankBlocks = kMaxK / 256;

__global__ void __launch_bounds__(256) topk_rank_count(const uint64_t *cand_key, const uint64_t *cand_idx,
                                                       int k, const TopkState *fast, unsigned int *partial) {
  const unsigned long long c = fast->ncand;
  if (c > (unsigned long long)kMaxK || c < (unsigned long long)k) return;
  const int n = (int)c;
  const int i0 = blockIdx.x * 256, j0 = blockIdx.y * 256;
  if (i0 >= n || j0 >= n) return;  // uniform over the block
  __shared__ uint64_t sk[256];
  __shared__ uint64_t si[256];
  const int t = threadIdx.x;
  // past the end: (key 0, index ~0), which never sorts before a candidate
  const bool live = j0 + t < n;
  sk[t] = live ? cand_key[j0 + t] : 0ull;
  si[t] = live ? cand_idx[j0 + t] : ~0ull;
  __syncthreads();
  const int i = i0 + t;
  if (i >= n) return;
  const uint64_t ki = cand_key[i], ii = cand_idx[i];
  unsigned int cnt = 0;
  // branch-free comparisons, several LDS reads in flight
#pragma unroll 16
  for (int j = 0; j < 256; ++j) {
    const uint64_t a = sk[j], b = si[j];
    cnt += (unsigned int)((a > ki) | ((a == ki) & (b < ii)));
  }
  partial[blockIdx.y * kMaxK + i] = cnt;
}

__global__ void __launch_bounds__(256) topk_rank_place(const uint64_t *cand_key, const uint64_t *cand_idx,
                                                       int k, int dtype, uint64_t *idx_out, double *val_out,
                                                       TopkState *fast, const unsigned int *partial) {
  const unsigned long long c = fast->ncand;
  if (c > (unsigned long long)kMaxK || c < (unsigned long long)k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fast->fallback = 1;
    return;
  }
  const int n = (int)c;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int nb = (n + 255) / 256;
  unsigned int r = 0;
  for (int b = 0; b < nb; ++b) r += partial[b * kMaxK + i];
  if (r < (unsigned int)k) {
    idx_out[r] = cand_idx[i];
    val_out[r] = key_value(cand_key[i], dtype);
  }
}

static void launch_rank_place(const uint64_t *cand_key, const uint64_t *cand_idx, int k, int dtype,
                              uint64_t *idx_out, double *val_out, TopkState *fast, unsigned int *partial,
                              hipStream_t s) {
  hipLaunchKernelGGL(topk_rank_count, dim3(kRankBlocks, kRankBlocks), dim3(256), 0, s, cand_key, cand_idx, k,
                     (const TopkState *)fast, partial);
  hipLaunchKernelGGL(topk_rank_place, dim3(kRankBlocks), dim3(256), 0, s, cand_key, cand_idx, k, dtype, idx_out,
                     val_out, fast, (const unsigned int *)partial);
}

// ---- fast path: per-chunk maxima bound the threshold from below
constexpr uint64_t kMaxChunk = 1ull << 13;

__global__ void __launch_bounds__(256) topk_chunk_max(const void *p, int dtype, uint64_t len,
                                                      uint64_t *cmax) {
  __shared__ uint64_t red[256];
  const uint64_t lo = blockIdx.x * kMaxChunk;
  const uint64_t hi = lo + kMaxChunk < len ? lo + kMaxChunk : len;
  uint64_t m = 0;
  if (dtype == 1 && hi - lo == kMaxChunk) {
    const float4 *v = (const float4 *)((const float *)p + lo);
#pragma unroll 4
    for (int i = threadIdx.x; i < (int)(kMaxChunk / 4); i += 256) {
      const float4 x = v[i];
      const float e[4] = {x.x, x.y, x.z, x.w};
      for (int t = 0; t < 4; ++t) {
        const uint32_t u = __float_as_uint(e[t]);
        const uint64_t key = (u & 0x80000000u) ? (uint64_t)(~u) : (uint64_t)(u | 0x80000000u);
        m = key > m ? key : m;
      }
    }
  } else {
    for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) {
      const uint64_t key = sort_key(p, dtype, i);
      m = key > m ? key : m;
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + w] ? red[threadIdx.x] : red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cmax[blockIdx.x] = red[0];
}

// every entry >= tau0 of the chunks whose maximum reaches tau0
__global__ void __launch_bounds__(256) topk_collect_fast(const void *p, int dtype, uint64_t len,
                                                         const uint64_t *cmax, const TopkState *sel,
                                                         TopkState *fast, uint64_t *cand_key,
                                                         uint64_t *cand_idx) {
  const uint64_t tau0 = sel->prefix;
  if (cmax[blockIdx.x] < tau0) return;
  const uint64_t lo = blockIdx.x * kMaxChunk;
  const uint64_t hi = lo + kMaxChunk < len ? lo + kMaxChunk : len;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const uint64_t key = sort_key(p, dtype, i);
    append_candidate(key >= tau0, key, i, fast, cand_key, cand_idx);
  }
}

// One launch sets up a fast form: its counters, the selection state over the
// chunk or tile maxima, the exact passes' state (used only if they run; the
// last selection pass leaves the histogram cleared for them) and the
// histogram.
__global__ void __launch_bounds__(256) topk_init_fast(TopkState *sel, TopkState *st, TopkState *fast,
                                                      unsigned long long *hist, int keybits, int k) {
  if (threadIdx.x == 0) {
    TopkState *both[2] = {sel, st};
    for (int i = 0; i < 2; ++i) {
      both[i]->prefix = 0;
      both[i]->hi_shift = keybits;
      both[i]->kr = (unsigned long long)k;
      both[i]->n_gt = 0;
    }
    fast->ncand = 0;
    fast->fallback = 0;
    fast->nq = 0;
  }
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
}

uint64_t topk_scratch_bytes(uint64_t len, int k) {
  const uint64_t nblocks = (len + kChunk - 1) / kChunk;
  const uint64_t nchunks = (len + kMaxChunk - 1) / kMaxChunk;
  return 3 * 256 + kBins * 8 + nblocks * 8 + nchunks * 8 + 2 * (uint64_t)kMaxK * 8 +
         2 * (uint64_t)k * 8 + (uint64_t)kRankBlocks * kMaxK * 4 + 1024;
}

// Exact passes over the whole vector: radix select of the k-th largest key,
// then the entries above it and the lowest-index entries equal to it.
static void exact_topk(const void *probs, int dtype, uint64_t len, int k, uint64_t *idx_out,
                       double *val_out, TopkState *st, unsigned long long *hist,
                       unsigned long long *blockcnt, uint64_t *cand_key, uint64_t *cand_idx,
                       const unsigned int *gate, hipStream_t s, bool initialized = false) {
  const uint64_t nblocks = (len + kChunk - 1) / kChunk;
  const int keybits = dtype == 1 ? 32 : 64;
  if (!initialized) hipLaunchKernelGGL(topk_init, dim3(1), dim3(256), 0, s, st, hist, keybits, k, gate);
  uint64_t hb = (len + 255) / 256;
  if (hb > kChunkGrid) hb = kChunkGrid;
  for (int resolved = 0; resolved < keybits;) {
    const int bits = (keybits - resolved) < kDigitBits ? (keybits - resolved) : kDigitBits;
    hipLaunchKernelGGL(topk_hist, dim3((unsigned)hb), dim3(256), 0, s, probs, dtype, len, st, hist, bits,
                       gate);
    hipLaunchKernelGGL(topk_select, dim3(1), dim3(256), 0, s, st, hist, bits, gate);
    resolved += bits;
  }
  const unsigned cg = (unsigned)(nblocks < kChunkGrid ? nblocks : kChunkGrid);
  hipLaunchKernelGGL(topk_collect_gt, dim3(cg), dim3(256), 0, s, probs, dtype, len, st, cand_key, cand_idx,
                     blockcnt, gate);
  hipLaunchKernelGGL(topk_scan, dim3(1), dim3(1024), 0, s, blockcnt, nblocks, gate);
  hipLaunchKernelGGL(topk_collect_eq, dim3(cg), dim3(256), 0, s, probs, dtype, len, st, k, cand_key, cand_idx,
                     blockcnt, gate);
  int npow = 1;
  while (npow < k) npow <<= 1;
  hipLaunchKernelGGL(topk_sort, dim3(1), dim3(1024), (size_t)16 * npow, s, cand_key, cand_idx, k, dtype, idx_out,
                     val_out, gate);
}

hipError_t launch_topk(const void *probs, int dtype, uint64_t len, int k, uint64_t *idx_out,
                       double *val_out, void *scratch, uint64_t scratch_bytes, hipStream_t s) {
  if (k < 1 || k > kMaxK || (uint64_t)k > len) return hipErrorInvalidValue;
  if (scratch_bytes < topk_scratch_bytes(len, k)) return hipErrorInvalidValue;
  char *sp = (char *)scratch;
  TopkState *st = (TopkState *)sp;          // exact passes
  TopkState *sel = (TopkState *)(sp + 256); // threshold over chunk maxima
  TopkState *fast = (TopkState *)(sp + 512);
  unsigned long long *hist = (unsigned long long *)(sp + 768);
  const uint64_t nblocks = (len + kChunk - 1) / kChunk;
  const uint64_t nchunks = (len + kMaxChunk - 1) / kMaxChunk;
  unsigned long long *blockcnt = hist + kBins;
  uint64_t *cmax = (uint64_t *)(blockcnt + nblocks);
  uint64_t *fkey = cmax + nchunks;
  uint64_t *fidx = fkey + kMaxK;
  uint64_t *cand_key = fidx + kMaxK;
  uint64_t *cand_idx = cand_key + k;
  unsigned int *partial = (unsigned int *)(cand_idx + k);
  const int keybits = dtype == 1 ? 32 : 64;
  if (nchunks < (uint64_t)k) {
    exact_topk(probs, dtype, len, k, idx_out, val_out, st, hist, blockcnt, cand_key, cand_idx,
               nullptr, s);
    return hipGetLastError();
  }
  // fast path: tau0 = k-th largest chunk maximum <= the k-th largest entry
  hipLaunchKernelGGL(topk_init_fast, dim3(1), dim3(256), 0, s, sel, st, fast, hist, keybits, k);
  hipLaunchKernelGGL(topk_chunk_max, dim3((unsigned)nchunks), dim3(256), 0, s, probs, dtype, len, cmax);
  uint64_t hb = (nchunks + 255) / 256;
  if (hb > 8192) hb = 8192;
  for (int resolved = 0; resolved < keybits;) {
    const int bits = (keybits - resolved) < kDigitBits ? (keybits - resolved) : kDigitBits;
    hipLaunchKernelGGL(topk_hist, dim3((unsigned)hb), dim3(256), 0, s, (const void *)cmax, 2, nchunks,
                       sel, hist, bits, (const unsigned int *)nullptr);
    hipLaunchKernelGGL(topk_select, dim3(1), dim3(256), 0, s, sel, hist, bits,
                       (const unsigned int *)nullptr);
    resolved += bits;
  }
  hipLaunchKernelGGL(topk_collect_fast, dim3((unsigned)nchunks), dim3(256), 0, s, probs, dtype, len,
                     cmax, sel, fast, fkey, fidx);
  launch_rank_place(fkey, fidx, k, dtype, idx_out, val_out, fast, partial, s);
  // exact passes, skipped on the device unless the fast path gave up
  exact_topk(probs, dtype, len, k, idx_out, val_out, st, hist, blockcnt, cand_key, cand_idx,
             &fast->fallback, s, true);
  return hipGetLastError();
}

// ---- fused form: the root contraction wrote, per output tile, the largest
// key of the values it stored.  The k-th largest tile maximum tau0 is a lower
// bound of the k-th largest entry (k tiles each hold an entry >= tau0), and
// every entry >= tau0 lies in a tile whose maximum reaches tau0, so only those
// tiles are gathered.  Tile t covers rows [tm*bm, tm*bm + bm) and columns
// [tn*bn, tn*bn + bn) of the root GEMM, t = tm * tilesN + tn; entry (m, n) is
// at output index deposit(m, posM) + deposit(n, posN).
// 1) list the tiles whose maximum reaches tau0 (more than kMaxK of them
//    means more than kMaxK candidates: mark the overflow instead)
__global__ void __launch_bounds__(256) topk_list_tiles(const unsigned long long *tkey, uint64_t ntiles,
                                                       const TopkState *sel, TopkState *fast,
                                                       uint64_t *qlist) {
  const uint64_t tau0 = sel->prefix;
  for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < ntiles; t += (uint64_t)gridDim.x * 256) {
    if (tkey[t] < tau0) continue;
    const unsigned long long q = atomicAdd(&fast->nq, 1ull);
    if (q < (unsigned long long)kMaxK) qlist[q] = t;
    else atomicAdd(&fast->ncand, (unsigned long long)kMaxK + 1);
  }
}

// 2) every entry >= tau0 of the listed tiles.  A block walks its share of
//    the list (grid-strided) with several loads in flight per thread,
//    stages its hits in LDS (one LDS atomic per wave and group of hits) and
//    reserves its slots in the global list with one atomic at the end; hits
//    past the kStage LDS slots go to the global list directly.  The stage is
//    small so that the kernel fits beside a running final-step kernel of
//    another stream (which leaves about 29 KB of a CU's LDS free).
constexpr int kCollectGrid = 1024;
constexpr int kCollectDepth = 16;  // float4 loads in flight per thread (vector form)
constexpr int kGenericDepth = 8;   // scalar loads in flight per thread (general form)
constexpr unsigned int kStage = 1024;

// every lane of the wave calls it
__device__ inline void stage_hit(bool hit, uint64_t key, uint64_t idx, unsigned int *bcount, uint64_t *bk,
                                 uint64_t *bi, TopkState *fast, uint64_t *cand_key, uint64_t *cand_idx) {
  const unsigned long long bal = __ballot(hit);
  if (!bal) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)bal) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(bcount, (unsigned int)__popcll(bal));
  base = __shfl(base, leader, 64);
  const unsigned int r = base + (unsigned int)__popcll(bal & ((1ull << lane) - 1ull));
  if (hit && r < kStage) {
    bk[r] = key;
    bi[r] = idx;
  }
  append_candidate(hit && r >= kStage, key, idx, fast, cand_key, cand_idx);
}

__global__ void __launch_bounds__(256) topk_collect_tiles(const void *p, int dtype, GemmArgs g, int lbm,
                                                          int lbn, uint64_t tilesN,
                                                          const uint64_t *qlist, const TopkState *sel,
                                                          TopkState *fast, uint64_t *cand_key,
                                                          uint64_t *cand_idx) {
  __shared__ uint64_t bk[kStage];
  __shared__ uint64_t bi[kStage];
  __shared__ unsigned int bcount;
  __shared__ unsigned long long bbase;
  const uint64_t tau0 = sel->prefix;
  const uint64_t nq = fast->nq < (unsigned long long)kMaxK ? fast->nq : (unsigned long long)kMaxK;
  const uint64_t M = 1ull << g.lm, N = 1ull << g.ln;
  if (threadIdx.x == 0) bcount = 0;
  __syncthreads();
  if (g.vec4 && g.ncompact == lbm + lbn && dtype == 1) {
    // full tile whose two lowest output bits are tile bits: compact index x
    // (tile entries in output order) lands at base + deposit(x, lpos), and
    // x, x+1, x+2, x+3 are adjacent in the output
    // x = r * 1024 + 4 * thread: the low 10 compact bits are fixed per
    // thread, the run r sets the rest (uniform over the block)
    const uint32_t runs4 = (1u << (lbm + lbn)) / 1024u;
    const int hb = lbm + lbn - 10;
    const uint64_t lo = deposit_c<10>((uint64_t)threadIdx.x * 4, g.lpos, 10);
    for (uint64_t q = blockIdx.x; q < nq; q += gridDim.x) {
      const uint64_t t = qlist[q];
      const uint64_t tm = t / tilesN, tn = t % tilesN;
      const uint64_t base =
          scatter_bits(tm << lbm, g.posM, g.lm) + scatter_bits(tn << lbn, g.posN, g.ln) + lo;
      for (uint32_t r0 = 0; r0 < runs4; r0 += kCollectDepth) {
        float4 v[kCollectDepth];
#pragma unroll
        for (int d = 0; d < kCollectDepth; ++d)
          if (r0 + d < runs4)
            v[d] = *(const float4 *)((const float *)p + base + deposit_c<6, 10>((uint64_t)(r0 + d), g.lpos, hb));
#pragma unroll
        for (int d = 0; d < kCollectDepth; ++d) {
          if (r0 + d < runs4) {  // uniform over the block
            const uint64_t at = base + deposit_c<6, 10>((uint64_t)(r0 + d), g.lpos, hb);
            const float e[4] = {v[d].x, v[d].y, v[d].z, v[d].w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const uint32_t u = __float_as_uint(e[c]);
              const uint64_t key = (u & 0x80000000u) ? (uint64_t)(~u) : (uint64_t)(u | 0x80000000u);
              stage_hit(key >= tau0, key, at + c, &bcount, bk, bi, fast, cand_key, cand_idx);
            }
          }
        }
      }
    }
  } else {
    const uint32_t runs = (1u << (lbm + lbn)) / 256u;  // tiles hold >= 1024 entries
    for (uint64_t q = blockIdx.x; q < nq; q += gridDim.x) {
      const uint64_t t = qlist[q];
      const uint64_t m0 = (t / tilesN) << lbm, n0 = (t % tilesN) << lbn;
      for (uint32_t r0 = 0; r0 < runs; r0 += kGenericDepth) {
        uint64_t key[kGenericDepth], at[kGenericDepth];
        bool ok[kGenericDepth];
#pragma unroll
        for (int d = 0; d < kGenericDepth; ++d) {
          const uint32_t e = (r0 + d) * 256u + threadIdx.x;
          const uint64_t rl = e >> lbn, cl = e & ((1u << lbn) - 1);
          ok[d] = r0 + d < runs && m0 + rl < M && n0 + cl < N;
          at[d] = ok[d] ? scatter_bits(m0 | rl, g.posM, g.lm) + scatter_bits(n0 | cl, g.posN, g.ln) : 0;
          key[d] = ok[d] ? sort_key(p, dtype, at[d]) : 0;
        }
#pragma unroll
        for (int d = 0; d < kGenericDepth; ++d)
          stage_hit(ok[d] && key[d] >= tau0, key[d], at[d], &bcount, bk, bi, fast, cand_key, cand_idx);
      }
    }
  }
  __syncthreads();
  const unsigned int kept = bcount < kStage ? bcount : kStage;
  if (kept == 0) return;  // uniform over the block
  if (threadIdx.x == 0) bbase = atomicAdd(&fast->ncand, (unsigned long long)kept);
  __syncthreads();
  const unsigned long long b0 = bbase;
  for (unsigned int i = threadIdx.x; i < kept; i += blockDim.x) {
    const unsigned long long slot = b0 + i;
    if (slot < (unsigned long long)kMaxK) {
      cand_key[slot] = bk[i];
      cand_idx[slot] = bi[i];
    }
  }
}

uint64_t topk_tiles_scratch_bytes(uint64_t len, uint64_t ntiles, int k) {
  const uint64_t nblocks = (len + kChunk - 1) / kChunk;
  (void)ntiles;
  return 3 * 256 + kBins * 8 + nblocks * 8 + 3 * (uint64_t)kMaxK * 8 + 2 * (uint64_t)k * 8 +
         (uint64_t)kRankBlocks * kMaxK * 4 + 1024;
}

hipError_t launch_topk_tiles(const void *probs, int dtype, uint64_t len, const GemmArgs &g, int lbm,
                             int lbn, const unsigned long long *tkey, uint64_t ntiles, int k,
                             uint64_t *idx_out, double *val_out, void *scratch, uint64_t scratch_bytes,
                             hipStream_t s) {
  if (k < 1 || k > kMaxK || (uint64_t)k > len) return hipErrorInvalidValue;
  if (scratch_bytes < topk_tiles_scratch_bytes(len, ntiles, k) || ntiles > 0x7fffffffull)
    return hipErrorInvalidValue;
  const uint64_t tilesN = ((1ull << g.ln) + (1ull << lbn) - 1) >> lbn;
  char *sp = (char *)scratch;
  TopkState *st = (TopkState *)sp;
  TopkState *sel = (TopkState *)(sp + 256);
  TopkState *fast = (TopkState *)(sp + 512);
  unsigned long long *hist = (unsigned long long *)(sp + 768);
  const uint64_t nblocks = (len + kChunk - 1) / kChunk;
  unsigned long long *blockcnt = hist + kBins;
  uint64_t *fkey = (uint64_t *)(blockcnt + nblocks);
  uint64_t *fidx = fkey + kMaxK;
  uint64_t *qlist = fidx + kMaxK;
  uint64_t *cand_key = qlist + kMaxK;
  uint64_t *cand_idx = cand_key + k;
  unsigned int *partial = (unsigned int *)(cand_idx + k);
  if (ntiles < (uint64_t)k) {
    exact_topk(probs, dtype, len, k, idx_out, val_out, st, hist, blockcnt, cand_key, cand_idx, nullptr, s);
    return hipGetLastError();
  }
  // float32 keys occupy the low 32 bits
  const int tbits = dtype == 1 ? 32 : 64;
  hipLaunchKernelGGL(topk_init_fast, dim3(1), dim3(256), 0, s, sel, st, fast, hist, tbits, k);
  uint64_t hb = (ntiles + 255) / 256;
  if (hb > 8192) hb = 8192;
  for (int resolved = 0; resolved < tbits;) {
    const int bits = (tbits - resolved) < kDigitBits ? (tbits - resolved) : kDigitBits;
    hipLaunchKernelGGL(topk_hist, dim3((unsigned)hb), dim3(256), 0, s, (const void *)tkey, 2, ntiles, sel,
                       hist, bits, (const unsigned int *)nullptr);
    hipLaunchKernelGGL(topk_select, dim3(1), dim3(256), 0, s, sel, hist, bits, (const unsigned int *)nullptr);
    resolved += bits;
  }
  uint64_t lg = (ntiles + 255) / 256;
  if (lg > 1024) lg = 1024;
  hipLaunchKernelGGL(topk_list_tiles, dim3((unsigned)lg), dim3(256), 0, s, tkey, ntiles, sel, fast, qlist);
  hipLaunchKernelGGL(topk_collect_tiles, dim3(kCollectGrid), dim3(256), 0, s, probs, dtype, g, lbm, lbn,
                     tilesN, (const uint64_t *)qlist, sel, fast, fkey, fidx);
  launch_rank_place(fkey, fidx, k, dtype, idx_out, val_out, fast, partial, s);
  exact_topk(probs, dtype, len, k, idx_out, val_out, st, hist, blockcnt, cand_key, cand_idx, &fast->fallback,
             s, true);
  return hipGetLastError();
}

// total of the per-tile float64 sums: block b adds the contiguous range
// [b*chunk, (b+1)*chunk) by a fixed strided split and a fixed tree, then one
// block adds the block partials the same way
constexpr int kSumBlocks = 256;

__device__ inline double block_sum_fixed(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(256) sum_tiles_pass1(const double *ts, uint64_t n, double *partial) {
  __shared__ double red[256];
  const uint64_t chunk = (n + kSumBlocks - 1) / kSumBlocks;
  const uint64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += 256) acc += ts[i];
  const double t = block_sum_fixed(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) sum_tiles_pass2(const double *partial, double *out) {
  __shared__ double red[256];
  const double t = block_sum_fixed(partial[threadIdx.x], red);
  if (threadIdx.x == 0) *out = t;
}

hipError_t launch_sum_tiles(const double *tsum, uint64_t ntiles, double *partial, double *out,
                            hipStream_t s) {
  hipLaunchKernelGGL(sum_tiles_pass1, dim3(kSumBlocks), dim3(256), 0, s, tsum, ntiles, partial);
  hipLaunchKernelGGL(sum_tiles_pass2, dim3(1), dim3(kSumBlocks), 0, s, (const double *)partial, out);
  return hipGetLastError();
}

// ============================================================= marginal
// out[y] = sum over x with bit keep[i] of x equal to bit i of y.
// Pass 1: block b owns the contiguous chunk [b*2^c, (b+1)*2^c); the kept
// bits below c give 2^rlo bins, each summed by a fixed set of threads in a
// fixed order, then combined by a fixed tree: partial[b][bin].
// Pass 2: out[y] = sum over the blocks whose kept high bits match y, in block
// order, by one block per y (fixed strided split + fixed tree).
struct MargArgs {
  const void *p;
  int dtype;
  int n, c;              // qubits, log2 chunk
  int rlo;               // kept bits below c
  int keep_lo_pos[24];   // address bit of bin bit i (kept, < c), bin bit i <-> y bit ylo_bit[i]
  int free_lo_pos[40];   // address bits < c that are summed, in increasing order
  int nfree_lo;
  int contig;            // no kept bit below c: the chunk is one bin, read linearly
  double *partial;
};

__device__ inline double load_prob(const void *p, int dtype, uint64_t i) {
  return dtype == 1 ? (double)((const float *)p)[i] : ((const double *)p)[i];
}

__global__ void __launch_bounds__(256) marg_pass1(MargArgs a) {
  __shared__ double red[256];
  const uint64_t base = (uint64_t)blockIdx.x << a.c;
  if (a.contig) {
    // one bin: every thread sums a fixed strided share with 16-byte loads
    const uint64_t n = 1ull << a.c;
    double s = 0.0;
    if (a.dtype == 1 && n >= 1024) {
      const float4 *v = (const float4 *)((const float *)a.p + base);
      for (uint64_t i = threadIdx.x; i < n / 4; i += 256) {
        const float4 x = v[i];
        s += ((double)x.x + (double)x.y) + ((double)x.z + (double)x.w);
      }
    } else if (a.dtype == 0 && n >= 512) {
      const double2 *v = (const double2 *)((const double *)a.p + base);
      for (uint64_t i = threadIdx.x; i < n / 2; i += 256) {
        const double2 x = v[i];
        s += x.x + x.y;
      }
    } else {
      for (uint64_t i = threadIdx.x; i < n; i += 256) s += load_prob(a.p, a.dtype, base + i);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
    return;
  }
  const int nbins = 1 << a.rlo;
  const uint64_t per_bin = 1ull << a.nfree_lo;
  for (int bin0 = 0; bin0 < nbins; bin0 += 256) {
    // threads per bin when bins < 256
    const int bins_here = (nbins - bin0) < 256 ? (nbins - bin0) : 256;
    const int tpb = 256 / bins_here;  // bins_here is a power of two
    const int bin = bin0 + (int)(threadIdx.x % bins_here);
    const int sub = (int)(threadIdx.x / bins_here);
    uint64_t boff = 0;
    for (int i = 0; i < a.rlo; ++i) boff |= (uint64_t)((bin >> i) & 1) << a.keep_lo_pos[i];
    double s = 0.0;
    if (sub < tpb) {
      for (uint64_t z = sub; z < per_bin; z += tpb) {
        uint64_t off = boff;
        for (int i = 0; i < a.nfree_lo; ++i) off |= ((z >> i) & 1ull) << a.free_lo_pos[i];
        s += load_prob(a.p, a.dtype, base + off);
      }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    // tree over the threads of each bin (threads bin + bins_here * sub)
    for (int w = tpb / 2; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w * bins_here) red[threadIdx.x] += red[threadIdx.x + w * bins_here];
      __syncthreads();
    }
    if ((int)threadIdx.x < bins_here)
      a.partial[(uint64_t)blockIdx.x * nbins + bin0 + threadIdx.x] = red[threadIdx.x];
    __syncthreads();
  }
}

struct Marg2Args {
  const double *partial;
  double *out;
  int rlo, rhi;
  int nblk_bits;               // log2 number of pass-1 blocks
  int keep_hi_blockbit[24];    // block-index bit of y's high kept bit j
  int free_hi_blockbit[40];    // block-index bits summed over, increasing
  int nfree_hi;
  int ylo_of_bin[24];          // y bit of bin bit i
  int yhi_bit[24];             // y bit of high kept bit j
};

__global__ void __launch_bounds__(256) marg_pass2(Marg2Args a) {
  __shared__ double red[256];
  const uint64_t y = blockIdx.x;
  uint64_t bin = 0;
  for (int i = 0; i < a.rlo; ++i) bin |= ((y >> a.ylo_of_bin[i]) & 1ull) << i;
  uint64_t bbase = 0;
  for (int j = 0; j < a.rhi; ++j) bbase |= ((y >> a.yhi_bit[j]) & 1ull) << a.keep_hi_blockbit[j];
  const uint64_t nsum = 1ull << a.nfree_hi;
  double s = 0.0;
  for (uint64_t w = threadIdx.x; w < nsum; w += 256) {
    uint64_t b = bbase;
    for (int i = 0; i < a.nfree_hi; ++i) b |= ((w >> i) & 1ull) << a.free_hi_blockbit[i];
    s += a.partial[(b << a.rlo) + bin];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.out[y] = red[0];
}

static int marg_chunk_bits(int n) { return n < 16 ? n : 16; }

uint64_t marginal_scratch_bytes(int n, int num_keep) {
  const int c = marg_chunk_bits(n);
  return (uint64_t)8 << (n - c + (num_keep < c ? num_keep : c));
}

hipError_t launch_marginal(const void *probs, int dtype, int n, int num_keep, const int *keep,
                           double *out, void *scratch, uint64_t scratch_bytes, hipStream_t s) {
  if (n < 0 || n > 40 || num_keep < 0 || num_keep > 24 || num_keep > n) return hipErrorInvalidValue;
  const int c = marg_chunk_bits(n);
  MargArgs a{};
  a.p = probs;
  a.dtype = dtype;
  a.n = n;
  a.c = c;
  int rlo = 0, nfl = 0;
  int ylo_of_bin[24], yhi_bit[24], keep_hi_blockbit[24];
  int rhi = 0;
  // kept address bits below c, in increasing address order
  for (int bit = 0; bit < n; ++bit) {
    int yi = -1;
    for (int i = 0; i < num_keep; ++i)
      if (keep[i] == bit) yi = i;
    if (bit < c) {
      if (yi >= 0) {
        a.keep_lo_pos[rlo] = bit;
        ylo_of_bin[rlo] = yi;
        ++rlo;
      } else {
        a.free_lo_pos[nfl++] = bit;
      }
    } else if (yi >= 0) {
      yhi_bit[rhi] = yi;
      keep_hi_blockbit[rhi] = bit - c;
      ++rhi;
    }
  }
  a.rlo = rlo;
  a.nfree_lo = nfl;
  a.contig = (rlo == 0) ? 1 : 0;
  for (int i = 0; i < nfl; ++i)
    if (a.free_lo_pos[i] != i) a.contig = 0;
  const uint64_t nblocks = 1ull << (n - c);
  if (scratch_bytes < (nblocks << rlo) * 8) return hipErrorInvalidValue;
  a.partial = (double *)scratch;
  hipLaunchKernelGGL(marg_pass1, dim3((unsigned)nblocks), dim3(256), 0, s, a);
  Marg2Args b{};
  b.partial = a.partial;
  b.out = out;
  b.rlo = rlo;
  b.rhi = rhi;
  b.nblk_bits = n - c;
  int nfh = 0;
  for (int bb = 0; bb < n - c; ++bb) {
    bool kept = false;
    for (int j = 0; j < rhi; ++j)
      if (keep_hi_blockbit[j] == bb) kept = true;
    if (!kept) b.free_hi_blockbit[nfh++] = bb;
  }
  b.nfree_hi = nfh;
  for (int i = 0; i < rlo; ++i) b.ylo_of_bin[i] = ylo_of_bin[i];
  for (int j = 0; j < rhi; ++j) {
    b.yhi_bit[j] = yhi_bit[j];
    b.keep_hi_blockbit[j] = keep_hi_blockbit[j];
  }
  hipLaunchKernelGGL(marg_pass2, dim3((unsigned)(1ull << num_keep)), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace tqc
