// Instantiations of the marginalisation kernels -- the survivor pass, the
// second half of the coefficient route and the posterior draws -- for one
// precision and one number of m groups (DOTPE_INST_PREC, DOTPE_INST_G).
// Their lanes evaluate the distance rule for many triples in a loop; this
// unit is compiled without machine-level loop-invariant hoisting, which
// would otherwise keep every FP64 constant of the rule (polynomial
// coefficients, table geometry) in a register pair for the whole kernel and
// halve the waves per SIMD.
#include <hip/hip_runtime.h>

#include "launch.h"

#ifndef DOTPE_INST_PREC
#error "DOTPE_INST_PREC must be defined"
#endif
#ifndef DOTPE_INST_G
#error "DOTPE_INST_G must be defined"
#endif

namespace dotpe {
namespace {

template <int PREC, int G>
hipError_t launch_marg(int mode, const FusedArgs& a, int64_t grid, hipStream_t s) {
  switch (mode) {
    case kSurvivors:
      if constexpr (PREC == kFP64) {
        return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((k_survivors<PREC, G>), dim3((unsigned)grid), dim3(256), 0, s, a);
        return hipGetLastError();
      }
    case kE2:
      hipLaunchKernelGGL((k_e2_tiles<PREC, G>), dim3((unsigned)grid), dim3(256), 0, s, a);
      return hipGetLastError();
    case kSample:
      hipLaunchKernelGGL((k_sample_tiles<PREC, G>), dim3((unsigned)grid), dim3(256), 0, s, a);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int PREC, int G>
hipError_t launch_marg_packed(int mode, const PackLaunch& p, hipStream_t s) {
  const dim3 grid((unsigned)p.off[p.n]);
  switch (mode) {
    case kSurvivors:
      if constexpr (PREC == kFP64) {
        return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((k_survivors_packed<PREC, G>), grid, dim3(256), 0, s, p);
        return hipGetLastError();
      }
    case kE2:
      hipLaunchKernelGGL((k_e2_tiles_packed<PREC, G>), grid, dim3(256), 0, s, p);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace

#define DOTPE_CAT4(a, b, c, d) a##b##c##d
#define DOTPE_NAME(P, G) DOTPE_CAT4(launch_marg_p, P, _g, G)

hipError_t DOTPE_NAME(DOTPE_INST_PREC, DOTPE_INST_G)(int mode, const FusedArgs& a, int64_t grid,
                                                     hipStream_t s) {
  return launch_marg<DOTPE_INST_PREC, DOTPE_INST_G>(mode, a, grid, s);
}

#define DOTPE_PNAME(P, G) DOTPE_CAT4(launch_marg_packed_p, P, _g, G)

hipError_t DOTPE_PNAME(DOTPE_INST_PREC, DOTPE_INST_G)(int mode, const PackLaunch& p,
                                                      hipStream_t s) {
  return launch_marg_packed<DOTPE_INST_PREC, DOTPE_INST_G>(mode, p, s);
}

}  // namespace dotpe
