// bf16 Legendre analysis kernel with 3 table plane(s) (see legendre_bf16.h);
// one translation unit per plane count and direction so that the six
// compile in parallel.
#include "legendre_bf16.h"

namespace sht {
namespace bf16p {
template hipError_t launch_analysis<3>(const BatchArgs&, float2*, float, hipStream_t);
}  // namespace bf16p
}  // namespace sht
