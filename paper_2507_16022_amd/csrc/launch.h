// Launchers of the fused likelihood kernel, one per (precision, number of m
// groups).  Each is compiled in its own translation units (fused_inst.hip and
// marg_inst.hip built with DOTPE_INST_PREC and DOTPE_INST_G), so the
// library's kernels compile in parallel; the host runtime picks one from the
// table below.
#pragma once

#include <hip/hip_runtime.h>

#include "bound.h"
#include "e2.h"
#include "fused.h"

namespace dotpe {

// mode: kEval, kPilot, kEvidence (the fast pass: fast must be true),
// kBound (split precisions; `grid` counts 128 x 128 tiles), kSurvivors
// (split precisions; workgroups of 4 waves that take the listed tiles in
// turn), kCoef or kE2 (the coefficient route: workgroups that take the
// chunk's work items in turn), kSample (posterior draws in the listed
// tiles, after kCoef over the same list).  Launches `grid` workgroups on stream s and
// returns the launch status.
typedef hipError_t (*FusedLaunchFn)(int mode, bool fast, const FusedArgs& a, int64_t grid,
                                    hipStream_t s);

#define DOTPE_FUSED_DECL(P, G)                                                              \
  hipError_t launch_fused_p##P##_g##G(int mode, bool fast, const FusedArgs& a, int64_t grid, \
                                      hipStream_t s);
DOTPE_FUSED_DECL(0, 1)
DOTPE_FUSED_DECL(0, 2)
DOTPE_FUSED_DECL(0, 3)
DOTPE_FUSED_DECL(0, 4)
DOTPE_FUSED_DECL(1, 1)
DOTPE_FUSED_DECL(1, 2)
DOTPE_FUSED_DECL(1, 3)
DOTPE_FUSED_DECL(1, 4)
DOTPE_FUSED_DECL(2, 1)
DOTPE_FUSED_DECL(2, 2)
DOTPE_FUSED_DECL(2, 3)
DOTPE_FUSED_DECL(2, 4)
#undef DOTPE_FUSED_DECL

// the survivor pass, kE2 and kSample (marg_inst.hip), called by the
// launchers above
#define DOTPE_MARG_DECL(P, G)                                                               \
  hipError_t launch_marg_p##P##_g##G(int mode, const FusedArgs& a, int64_t grid, hipStream_t s);
DOTPE_MARG_DECL(0, 1)
DOTPE_MARG_DECL(0, 2)
DOTPE_MARG_DECL(0, 3)
DOTPE_MARG_DECL(0, 4)
DOTPE_MARG_DECL(1, 1)
DOTPE_MARG_DECL(1, 2)
DOTPE_MARG_DECL(1, 3)
DOTPE_MARG_DECL(1, 4)
DOTPE_MARG_DECL(2, 1)
DOTPE_MARG_DECL(2, 2)
DOTPE_MARG_DECL(2, 3)
DOTPE_MARG_DECL(2, 4)
#undef DOTPE_MARG_DECL

// Packed launches (pack.h): mode kPilot, kEvidence (the fast pass), kBound,
// kSurvivors, kCoef or kE2 for the events of p, grid p.off[p.n]; n_phi is
// the largest phase count among them (it sizes the fused kernel's LDS).
typedef hipError_t (*PackedLaunchFn)(int mode, const PackLaunch& p, int n_phi, hipStream_t s);

#define DOTPE_PACKED_DECL(P, G)                                                            \
  hipError_t launch_packed_p##P##_g##G(int mode, const PackLaunch& p, int n_phi, hipStream_t s); \
  hipError_t launch_marg_packed_p##P##_g##G(int mode, const PackLaunch& p, hipStream_t s);
DOTPE_PACKED_DECL(0, 1)
DOTPE_PACKED_DECL(0, 2)
DOTPE_PACKED_DECL(0, 3)
DOTPE_PACKED_DECL(0, 4)
DOTPE_PACKED_DECL(1, 1)
DOTPE_PACKED_DECL(1, 2)
DOTPE_PACKED_DECL(1, 3)
DOTPE_PACKED_DECL(1, 4)
DOTPE_PACKED_DECL(2, 1)
DOTPE_PACKED_DECL(2, 2)
DOTPE_PACKED_DECL(2, 3)
DOTPE_PACKED_DECL(2, 4)
#undef DOTPE_PACKED_DECL

inline PackedLaunchFn packed_launcher(int prec, int G) {
  static const PackedLaunchFn table[3][kMaxG] = {
      {launch_packed_p0_g1, launch_packed_p0_g2, launch_packed_p0_g3, launch_packed_p0_g4},
      {launch_packed_p1_g1, launch_packed_p1_g2, launch_packed_p1_g3, launch_packed_p1_g4},
      {launch_packed_p2_g1, launch_packed_p2_g2, launch_packed_p2_g3, launch_packed_p2_g4}};
  if (prec < 0 || prec > 2 || G < 1 || G > kMaxG) return nullptr;
  return table[prec][G - 1];
}

// launcher for precision prec (kFP64, kFP16X2, kBF16X2) and G m groups
// (1..kMaxG), or nullptr
inline FusedLaunchFn fused_launcher(int prec, int G) {
  static const FusedLaunchFn table[3][kMaxG] = {
      {launch_fused_p0_g1, launch_fused_p0_g2, launch_fused_p0_g3, launch_fused_p0_g4},
      {launch_fused_p1_g1, launch_fused_p1_g2, launch_fused_p1_g3, launch_fused_p1_g4},
      {launch_fused_p2_g1, launch_fused_p2_g2, launch_fused_p2_g3, launch_fused_p2_g4}};
  if (prec < 0 || prec > 2 || G < 1 || G > kMaxG) return nullptr;
  return table[prec][G - 1];
}

}  // namespace dotpe
