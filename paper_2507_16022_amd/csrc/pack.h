// pack.h -- several events' work in one launch.
//
// A packed launch runs one pass of the evidence path (pilot, fast pass,
// bound pass, survivor pass, or one chunk of the coefficient route) for up to
// kMaxPack events at once.  Each event keeps the workgroup grid it would be
// launched with alone; the grids are laid end to end, each starting at a
// multiple of 8 so that an event's workgroups keep the XCD (blockIdx mod 8)
// the band raster of its tiles assumes.  A workgroup finds its event by the
// offsets, reads the event's arguments from device memory and runs the same
// tile code with its index within that event's grid.
#pragma once

#include "common.h"

namespace dotpe {

struct FusedArgs;

constexpr int kMaxPack = 16;

// the pointer arguments of one event (a kernel's pointer arguments are known
// to address global memory, so its loads and stores through them are global
// ones; pointers read from device memory would be generic, and their
// accesses flat ones)
struct PackPtrs {
  const int64_t* sub_idx;
  const void* B0;
  const void* B1;
  const void* B2;
  const void* B3;
  const double* col_scale;
  const double* ln_w_ext;
  const void* Ah0;
  const void* Ah1;
  const double* ah_scale;
  const void* Bh0;
  const void* Bh1;
  const double* bh_scale;
  const double* phase_cs;
  uint64_t* state;
  double* partials;
  double* cand;
  int* rerun;
  uint16_t* surv;
  int* surv_list;
  const float2* b_nrm;
  const float2* ah_nrm;
  const float2* bh_nrm;
  void* coef;
  double* rowcol;
};

struct PackLaunch {
  const FusedArgs* args;        // device: the batch's per-event arguments (sizes, tables)
  int64_t chunk;                // coefficient route: work0 = chunk * coef_tiles
  int n;                        // events in this launch, 1..kMaxPack
  int ev[kMaxPack];             // index into args of each
  int64_t off[kMaxPack + 1];    // first workgroup of each (multiples of 8); off[n] = grid
  // pointers of the bank and the context (the same for every event)
  const void* A0;
  const void* A1;
  const void* R0;
  const void* R1;
  const double* row_scale;
  const double* ln_w_bank;
  const float2* a_nrm;
  const double* dist_tab;
  const DistParams* dist_prm;
  PackPtrs ptr[kMaxPack];       // pointers of each event
};
static_assert(sizeof(PackLaunch) <= 4096, "packed launch arguments fit the kernel-argument limit");

// the event of workgroup g, its slot in the launch (*slot), and g's index and
// grid within it (static indices only, so the kernel-argument arrays are
// read by scalar loads)
__device__ __forceinline__ int pack_locate(const PackLaunch& p, int64_t g, int64_t* blk,
                                           int64_t* nblk, int* slot) {
  int e = p.ev[0], q = 0;
  int64_t o0 = 0, o1 = p.off[1];
#pragma unroll
  for (int k = 1; k < kMaxPack; ++k) {
    if (k < p.n && g >= p.off[k]) {
      e = p.ev[k];
      q = k;
      o0 = p.off[k];
      o1 = p.off[k + 1];
    }
  }
  *blk = g - o0;
  *nblk = o1 - o0;
  *slot = q;
  return e;
}

}  // namespace dotpe
