// Single-precision storage forms (FP32, BF16X3) of the contractions.  The
// matrix-core kernels for these forms are not part of this build yet: the
// entry points reject them with LRDM_EUNSUPPORTED before any launch, and these
// definitions only complete the template set.
#include "lrdm_internal.h"

namespace lrdm {

template <>
hipError_t launch_tn_sym<float>(lrdm_ctx*, const float*, const float*, const double*, int64_t, int,
                                int64_t, int, int, lrdm_prec, double*) {
  return hipErrorNotSupported;
}

template <>
hipError_t launch_backproj<float>(lrdm_ctx*, const float*, const double*, int, int64_t, int, int,
                                  lrdm_prec, double, const double*, double*) {
  return hipErrorNotSupported;
}

template <>
hipError_t launch_nn<float>(lrdm_ctx*, const double*, const float*, float*, int, int64_t) {
  return hipErrorNotSupported;
}

template <>
lrdm_status rayleigh_ritz<float>(lrdm_ctx* ctx, const Grid3&, const double*, float*, int, lrdm_prec,
                                 double*) {
  ctx->err = "single-precision Rayleigh-Ritz is not available in this build";
  return LRDM_EUNSUPPORTED;
}

}  // namespace lrdm
