// Float32 Legendre kernels with 2 field groups per workgroup (see
// legendre.h); one translation unit per NCB so that they compile in parallel.
#include "legendre.h"

namespace sht {
namespace fp32k {
template hipError_t launch_ncb<2>(bool, const BatchArgs&, const float2*, float2*, float, hipStream_t);
}  // namespace fp32k
}  // namespace sht
