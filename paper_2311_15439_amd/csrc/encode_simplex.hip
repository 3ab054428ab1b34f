// Simplex-cell instantiation of the encoding kernels (the paper's method).
#include "encode_dispatch.hpp"

namespace spx {
hipError_t encode_simplex(const EncodeCall& c) { return dispatch_D<SimplexTag>(c); }
}  // namespace spx
