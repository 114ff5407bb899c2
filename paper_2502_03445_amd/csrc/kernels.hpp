// Host-callable launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace tqc {

// operand exponents e_j of m leaves from their abs-max bits, and the output
// scale 2^(-K - sum e_j)
struct ScaleRec {
  const unsigned long long *maxbits;
  int m, K;
  int *exps;
  double *root_scale;
};

hipError_t launch_transform(const TransformArgs &a, hipStream_t s);
hipError_t launch_transforms(const TransformArgs *args, int n, hipStream_t s);  // n tensors
hipError_t launch_pack(const PackArgs &a, hipStream_t s);
hipError_t launch_f64_to_f32(const double *in, float *out, uint64_t n, hipStream_t s);
hipError_t launch_scale_f64(double *buf, uint64_t n, double sc, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *buf, uint64_t n, hipStream_t s);
// out[0] = bits of max |a - ref|, out[1] = bits of max |ref| (out cleared first)
hipError_t launch_max_abs_diff(const void *a, int a_f32, const double *ref, uint64_t n, unsigned long long *out,
                               hipStream_t s);
hipError_t launch_stamp(unsigned long long *dst, hipStream_t s);
hipError_t launch_f16_split(const float *src0, uint64_t n0, uint16_t *hi0, uint16_t *lo0, const float *src1,
                            uint64_t n1, uint16_t *hi1, uint16_t *lo1, unsigned long long *maxbits,
                            const double *root_scale, double *root_scale2, hipStream_t s);
uint64_t colnorm_scratch_entries(uint64_t rows, uint64_t cols);
hipError_t launch_column_norms(const double *T, uint64_t rows, uint64_t cols, double *partial, double *norms,
                               hipStream_t s);
hipError_t launch_gather_columns(const double *src, uint64_t rows, uint64_t src_cols, const int32_t *states,
                                 uint64_t count, uint64_t dst_cols, double *dst, hipStream_t s);
// n passes; the first launch's first workgroup clears zero[0 .. nzero) first
hipError_t launch_transform_passes(const TransformPassArgs *args, int n, hipStream_t s,
                                   unsigned long long *zero = nullptr, int nzero = 0);
// np (<= kPassBatch) passes of one level and nt (<= 4) per-entry transforms
// of other tensors in one launch
hipError_t launch_transform_level(const TransformPassArgs *pa, int np, const TransformArgs *ta, int nt,
                                  hipStream_t s);
// n leaves; with sr, the first launch's first thread also writes its
// exponents and output scale (for packs that read the abs-max directly)
hipError_t launch_packs(const PackArgs *args, int n, hipStream_t s, const ScaleRec *sr = nullptr);
int root_gemm_warm();  // caches the device's CU count (call outside graph capture)
hipError_t launch_absmax(const AbsMaxArgs *args, int n, hipStream_t s);                  // n leaves
// prec: 0 f64, 1 f32, 2 bf16x3, 3 bf16x6; tile: 0 = 128x128, 1 = 64x64, 2 = 32x32
// general = true: the general kernel even where the long-k kernel applies
hipError_t launch_gemm(int prec, const GemmArgs &g, int tile, hipStream_t s, bool general = false);
// long-k steps (k >= 512; k >= 256 in float64) on 128 x 128 tiles, at least min_tiles of them:
// the kernel with a deep LDS ring of operand slices (same results as
// launch_gemm's general kernel)
bool gemm_long_eligible(int prec, const GemmArgs &g, uint64_t min_tiles);
hipError_t launch_gemm_long(int prec, const GemmArgs &g, hipStream_t s);
// persistent final-step GEMM (128 x 128 tiles, K <= 256, float32 output in a
// layout whose two lowest output bits fall in every tile); hipErrorNotSupported
// when the step does not qualify
bool root_gemm_eligible(int prec, const GemmArgs &g);
hipError_t launch_root_gemm(int prec, const GemmArgs &g, hipStream_t s);
// the persistent final step of many reconstructions in one launch: one
// record per job (arguments prepared for 128 x 128 tiles, tile counts),
// all of one form and one kpad (4..8), each job eligible as above;
// blocks_per_job workgroups per job (a multiple of 8), jobs on grid y
struct RootJob {
  GemmArgs g;
  uint32_t ntiles;
  int lgtm, lgtn;
};
RootJob make_root_job(int prec, const GemmArgs &g);
hipError_t launch_root_multi(int prec, int kpad, const RootJob *jobs, int njobs, int blocks_per_job,
                             hipStream_t s);

// grouped launches: one launch runs the same kind of work of many
// reconstructions.  Record r owns workgroups [first[r], first[r + 1]) of the
// grid (first: device array of n + 1 entries, first[0] = 0, increasing; the
// grid has first[n] workgroups) and runs them as workgroups 0.. of its own
// launch of first[r + 1] - first[r] workgroups would.  The *_blocks helpers
// give the workgroup count of a record's own launch.
struct ZeroRec {
  unsigned long long *p;
  uint64_t n;
};
uint32_t grouped_pass_blocks(const TransformPassArgs &a);
uint32_t grouped_transform_blocks(const TransformArgs &a);
uint32_t grouped_absmax_blocks(const AbsMaxArgs &a);
uint32_t grouped_pack_blocks(const PackArgs &a);
hipError_t launch_grouped_passes(const TransformPassArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                 hipStream_t s);
hipError_t launch_grouped_transforms(const TransformArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                     hipStream_t s);
hipError_t launch_grouped_zero(const ZeroRec *recs, int n, hipStream_t s);   // one workgroup per record
hipError_t launch_grouped_absmax(const AbsMaxArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                                 hipStream_t s);
hipError_t launch_grouped_scales(const ScaleRec *recs, int n, hipStream_t s);  // one thread per record
hipError_t launch_grouped_packs(const PackArgs *recs, const uint32_t *first, int n, uint32_t blocks, hipStream_t s);
// the kernel variant launch_gemm picks for a step (tile, k step, float64
// folding, split count); grouped GEMM records are prepared for the tile
// (prepare_gemm_args) and must not split
struct GemmClass {
  int prec, tile, bk, ksplit;
  bool a64;
  uint64_t tiles;
  bool operator<(const GemmClass &o) const {
    if (prec != o.prec) return prec < o.prec;
    if (tile != o.tile) return tile < o.tile;
    if (bk != o.bk) return bk < o.bk;
    return a64 < o.a64;
  }
};
GemmClass gemm_class(int prec, const GemmArgs &g, int tile);
hipError_t launch_grouped_gemm(const GemmClass &c, const GemmArgs *recs, const uint32_t *first, int n, uint32_t blocks,
                               hipStream_t s);

// output forms
hipError_t launch_topk(const void *probs, int dtype, uint64_t len, int k, uint64_t *idx_out,
                       double *val_out, void *scratch, uint64_t scratch_bytes, hipStream_t s);
uint64_t topk_scratch_bytes(uint64_t len, int k);
hipError_t launch_marginal(const void *probs, int dtype, int n, int num_keep, const int *keep,
                           double *out, void *scratch, uint64_t scratch_bytes, hipStream_t s);
uint64_t marginal_scratch_bytes(int n, int num_keep);
// fused forms over the per-tile statistics of a root GEMM (tiles of
// 2^lbm x 2^lbn, see GemmArgs::tkey / tsum)
uint64_t topk_tiles_scratch_bytes(uint64_t len, uint64_t ntiles, int k);
hipError_t launch_topk_tiles(const void *probs, int dtype, uint64_t len, const GemmArgs &g, int lbm,
                             int lbn, const unsigned long long *tkey, uint64_t ntiles, int k,
                             uint64_t *idx_out, double *val_out, void *scratch, uint64_t scratch_bytes,
                             hipStream_t s);
// partial: 256 doubles of device scratch
hipError_t launch_sum_tiles(const double *tsum, uint64_t ntiles, double *partial, double *out,
                            hipStream_t s);

}  // namespace tqc
