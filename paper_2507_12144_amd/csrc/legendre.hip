// Entry points of the float32 Legendre contraction (kernels in
// legendre.h, instantiated per NCB in legendre_ncb{2,3,4}.hip).
#include "legendre.h"

namespace sht {
namespace {

using fp32k::launch_ncb;

hipError_t launch_fp32(bool analysis, const BatchArgs& b, const float2* in, float2* out, float c_rest,
                       hipStream_t st) {
  switch (b.ncb) {
    case 2: return launch_ncb<2>(analysis, b, in, out, c_rest, st);
    case 3: return launch_ncb<3>(analysis, b, in, out, c_rest, st);
    case 4: return launch_ncb<4>(analysis, b, in, out, c_rest, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int legendre_ring_pad(int nk) {
  const int ks[] = {16, 32, 48, 64, 96};
  for (int k : ks)
    if (4 * k >= nk) return 4 * k;
  return -1;
}

bool legendre_ncb_supported(int ncb) { return ncb >= 2 && ncb <= 4; }

hipError_t launch_legendre_analysis_batched(const BatchArgs& b, float2* y, float c_rest, hipStream_t st) {
  return launch_fp32(true, b, nullptr, y, c_rest, st);
}

hipError_t launch_legendre_synthesis_batched(const BatchArgs& b, const float2* y, hipStream_t st) {
  return launch_fp32(false, b, y, nullptr, 1.f, st);
}

}  // namespace sht
