// Instantiations of the fused likelihood kernel and the bound pass for one
// precision and one number of m groups, chosen at compile time by
// DOTPE_INST_PREC (0 FP64, 1 FP16x2, 2 BF16x2) and DOTPE_INST_G (1..4).  The
// marginalisation kernels of the same pair are in marg_inst.hip.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

#ifndef DOTPE_INST_PREC
#error "DOTPE_INST_PREC must be defined"
#endif
#ifndef DOTPE_INST_G
#error "DOTPE_INST_G must be defined"
#endif

namespace dotpe {

#define DOTPE_MARG_CAT4(a, b, c, d) a##b##c##d
#define DOTPE_MARG_NAME(P, G) DOTPE_MARG_CAT4(launch_marg_p, P, _g, G)
#define DOTPE_MARGP_NAME(P, G) DOTPE_MARG_CAT4(launch_marg_packed_p, P, _g, G)

namespace {

template <int PREC, int G, int MODE, bool FAST>
hipError_t launch_one(const FusedArgs& a, int64_t grid, hipStream_t s) {
  typedef Tile<PREC> TL;
  const size_t sh = TL::CS_OFF + sizeof(double) * kMaxM * a.n_phi * 2;
  // allow more than 64 KiB of dynamic LDS (once per kernel; not every
  // runtime needs or supports the attribute, so a failure is not an error)
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    const size_t most = TL::CS_OFF + sizeof(double) * kMaxM * kMaxPhi * 2;
    if (hipFuncSetAttribute((const void*)k_lnl_fused<PREC, G, MODE, FAST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
      (void)hipGetLastError();
  });
  hipLaunchKernelGGL((k_lnl_fused<PREC, G, MODE, FAST>), dim3((unsigned)grid), dim3(TL::NT), sh, s,
                     a);
  return hipGetLastError();
}

template <int PREC, int G>
hipError_t launch_bound(const FusedArgs& a, int64_t grid, hipStream_t s) {
  if constexpr (PREC == kFP64) {
    return hipErrorInvalidValue;
  } else {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      if (hipFuncSetAttribute((const void*)k_lnl_bound<PREC, G>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              BoundTile::LDS_BYTES) != hipSuccess)
        (void)hipGetLastError();
    });
    hipLaunchKernelGGL((k_lnl_bound<PREC, G>), dim3((unsigned)grid), dim3(BoundTile::NT),
                       BoundTile::LDS_BYTES, s, a);
    return hipGetLastError();
  }
}

template <int PREC, int G, int MODE, bool FAST>
hipError_t launch_one_packed(const PackLaunch& p, int n_phi, hipStream_t s) {
  typedef Tile<PREC> TL;
  const size_t sh = TL::CS_OFF + sizeof(double) * kMaxM * n_phi * 2;
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    const size_t most = TL::CS_OFF + sizeof(double) * kMaxM * kMaxPhi * 2;
    if (hipFuncSetAttribute((const void*)k_lnl_fused_packed<PREC, G, MODE, FAST>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)most) != hipSuccess)
      (void)hipGetLastError();
  });
  hipLaunchKernelGGL((k_lnl_fused_packed<PREC, G, MODE, FAST>), dim3((unsigned)p.off[p.n]),
                     dim3(TL::NT), sh, s, p);
  return hipGetLastError();
}

template <int PREC, int G>
hipError_t launch_bound_packed(const PackLaunch& p, hipStream_t s) {
  if constexpr (PREC == kFP64) {
    return hipErrorInvalidValue;
  } else {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      if (hipFuncSetAttribute((const void*)k_lnl_bound_packed<PREC, G>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              BoundTile::LDS_BYTES) != hipSuccess)
        (void)hipGetLastError();
    });
    hipLaunchKernelGGL((k_lnl_bound_packed<PREC, G>), dim3((unsigned)p.off[p.n]),
                       dim3(BoundTile::NT), BoundTile::LDS_BYTES, s, p);
    return hipGetLastError();
  }
}

template <int PREC, int G>
hipError_t launch_any_packed(int mode, const PackLaunch& p, int n_phi, hipStream_t s) {
  if (p.n < 1 || p.n > kMaxPack || p.off[p.n] <= 0) return hipErrorInvalidValue;
  switch (mode) {
    case kPilot: return launch_one_packed<PREC, G, kPilot, false>(p, n_phi, s);
    case kEvidence: return launch_one_packed<PREC, G, kEvidence, true>(p, n_phi, s);
    case kBound: return launch_bound_packed<PREC, G>(p, s);
    case kCoef: return launch_one_packed<PREC, G, kCoef, false>(p, n_phi, s);
    case kSurvivors:
    case kE2: return DOTPE_MARGP_NAME(DOTPE_INST_PREC, DOTPE_INST_G)(mode, p, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int G>
hipError_t launch_any(int mode, bool fast, const FusedArgs& a, int64_t grid, hipStream_t s) {
  switch (mode) {
    case kEval: return launch_one<PREC, G, kEval, false>(a, grid, s);
    case kPilot: return launch_one<PREC, G, kPilot, false>(a, grid, s);
    case kEvidence:
      // only the fast pass: without the cut every tile takes the
      // coefficient route
      return fast ? launch_one<PREC, G, kEvidence, true>(a, grid, s) : hipErrorInvalidValue;
    case kBound: return launch_bound<PREC, G>(a, grid, s);
    case kCoef: return launch_one<PREC, G, kCoef, false>(a, grid, s);
    case kSurvivors:
    case kE2:
    case kSample: return DOTPE_MARG_NAME(DOTPE_INST_PREC, DOTPE_INST_G)(mode, a, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

#define DOTPE_CAT4(a, b, c, d) a##b##c##d
#define DOTPE_NAME(P, G) DOTPE_CAT4(launch_fused_p, P, _g, G)

hipError_t DOTPE_NAME(DOTPE_INST_PREC, DOTPE_INST_G)(int mode, bool fast, const FusedArgs& a,
                                                     int64_t grid, hipStream_t s) {
  return launch_any<DOTPE_INST_PREC, DOTPE_INST_G>(mode, fast, a, grid, s);
}

#define DOTPE_PNAME(P, G) DOTPE_CAT4(launch_packed_p, P, _g, G)

hipError_t DOTPE_PNAME(DOTPE_INST_PREC, DOTPE_INST_G)(int mode, const PackLaunch& p, int n_phi,
                                                      hipStream_t s) {
  return launch_any_packed<DOTPE_INST_PREC, DOTPE_INST_G>(mode, p, n_phi, s);
}

}  // namespace dotpe
