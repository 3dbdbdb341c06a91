// bf16 Legendre kernels with 3 table plane(s) (see legendre_bf16.h); one
// translation unit per plane count so that the three compile in parallel.
#include "legendre_bf16.h"

namespace sht {
namespace bf16p {
template hipError_t launch_batched<3>(bool, const BatchArgs&, const void*, void*, float, hipStream_t);
}  // namespace bf16p
}  // namespace sht
