// Entry points of the bf16 Legendre forms (kernels in legendre_bf16.h,
// instantiated per plane count and direction in
// legendre_bf16_np{1,2,3}_{ana,syn}.hip).
#include "legendre_bf16.h"

namespace sht {

hipError_t launch_legendre_analysis_bf16_batched(const BatchArgs& b, int planes, float2* y, float c_rest,
                                                 hipStream_t st) {
  switch (planes) {
    case 1: return bf16p::launch_analysis<1>(b, y, c_rest, st);
    case 2: return bf16p::launch_analysis<2>(b, y, c_rest, st);
    case 3: return bf16p::launch_analysis<3>(b, y, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_legendre_synthesis_bf16_batched(const BatchArgs& b, int planes, const float2* y, hipStream_t st) {
  switch (planes) {
    case 1: return bf16p::launch_synthesis<1>(b, y, st);
    case 2: return bf16p::launch_synthesis<2>(b, y, st);
    case 3: return bf16p::launch_synthesis<3>(b, y, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sht
