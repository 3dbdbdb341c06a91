// bf16 Legendre synthesis kernel with 1 table plane(s) (see legendre_bf16.h);
// one translation unit per plane count and direction so that the six
// compile in parallel.
#include "legendre_bf16.h"

namespace sht {
namespace bf16p {
template hipError_t launch_synthesis<1>(const BatchArgs&, const float2*, hipStream_t);
}  // namespace bf16p
}  // namespace sht
