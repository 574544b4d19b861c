// pivot.h -- launch interface of the pivot-based counting kernel.
#pragma once

#include "internal.h"

// One launch over roots[0 .. nroots) (ranks, all of one bitmap width).
struct PivParams {
  const int32_t* dptr;
  const int32_t* dcol;
  const int32_t* orig;
  const int32_t* roots;
  const u64* gw;
  int kmax;              // counts for k = 2 .. kmax (<= 63)
  int fingerprint;
  int32_t nroots;
  int32_t drows;
  unsigned* cursor;
  u64* stack;            // per wave: pivot_stack_words(W, kmax, drows) words
  const u64* binom;      // C(n, r) table (n <= 1024, r <= 16; 2 words each), or null
  u64* wave_out;         // per wave: 256 words (3 per k, then counters)
  int* abort_flag;
  u64 deadline;          // wall_clock64 ticks from the launch; 0 = none
  u64* per_root;         // optional: 3 words per input id, for k = per_root_k
  int per_root_k;
  int nsub;              // work units per root (>= 1): unit s of a root takes
                         // the tree nodes at depth split_depth whose entry
                         // number is s mod nsub (and, for s = 0, the leaves
                         // above that depth)
  int split_depth;       // >= 1
};

int pivot_launch(int W, const PivParams& prm, int grid, size_t lds, hipStream_t s);
int pivot_occupancy(int W, size_t lds);
size_t pivot_lds_bytes(int W, int fp, int drows);
// Stack words per wave: frames of 3 W + kmax + 1 words (P, R, D, the pivot
// polynomial) and 4 scalar words for depths 0 .. drows + 1.
__host__ __device__ inline size_t pivot_stack_words(int W, int kmax, int drows) {
  const size_t fw = (size_t)3 * W + (size_t)(kmax + 1);
  return (size_t)(drows + 2) * (fw + 4);
}
