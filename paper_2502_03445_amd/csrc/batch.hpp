// Work-queue descriptors of the persistent batch kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace tqc {

enum UnitKind : int { UNIT_TRANSFORM = 0, UNIT_PACK = 1, UNIT_GEMM = 2 };

struct BatchUnit {
  int kind;
  int job;
  int dep0, dep1;    // units that must be complete first (-1: none)
  int arg;           // index into the kind's argument array
  int tile;          // GEMM tile id (0: 128x128, 1: 64x64, 2: 32x32)
  int is_root;       // completing this unit completes its job
  int pad;
  uint64_t first;    // global index of the unit's first item
  uint64_t ntiles;   // items of this unit
};

struct BatchDesc {
  const BatchUnit *units;
  int nunits;
  const TransformArgs *targs;
  const PackArgs *pargs;
  const GemmArgs *gargs;
  unsigned int *counters;         // finished items per unit
  unsigned long long *next;       // next item to claim
  unsigned long long total;       // number of items
  unsigned long long *job_start;  // device wall clock of a job's first item
  unsigned long long *job_end;    // ... and of its last
  unsigned int *error;            // set when a wait exceeded spin_limit
  unsigned long long spin_limit;
  // pre-pass (one launch each over all jobs): Pauli transform of raw
  // tensors, per-leaf largest |value|, per-job power-of-two exponents
  int ntransforms;
  uint64_t max_transform_elems;
  const AbsMaxArgs *aargs;
  int nleaves;
  uint64_t max_leaf_elems;
  unsigned long long *maxbits;    // per leaf (all jobs)
  int *exps;                      // per leaf
  double *root_scale;             // per job
  const int *job_leaf0;           // first leaf of each job (njobs + 1 entries)
  const int *job_cuts;            // K of each job
  int nowait;                     // 1: items of one launch never depend on each other
  unsigned long long first_item;  // this launch claims items [first_item, total)
  int nlevels;
  const unsigned long long *level_first;  // host array: item range of each level
};

// level_first: nlevels + 1 item offsets (host memory).  levels = 0: one
// launch with dependency waits; levels = 1: one launch per level, no waits.
hipError_t launch_batch(int prec, const BatchDesc &d, int njobs, int grid, int by_level,
                        hipStream_t s);
int batch_blocks_per_cu(int prec);

}  // namespace tqc
