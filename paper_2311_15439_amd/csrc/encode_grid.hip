// 2^n-corner grid instantiation of the encoding kernels (the baseline).
#include "encode_dispatch.hpp"

namespace spx {
hipError_t encode_grid(const EncodeCall& c) { return dispatch_D<GridTag>(c); }
}  // namespace spx
