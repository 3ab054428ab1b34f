// One (cell, dimension, feature count) instantiation of the encoding
// kernels.  The build compiles this file once per triple with SPX_UNIT_GRID
// (0: simplex cell, the paper's method; 1: the 2^n-corner grid baseline),
// SPX_UNIT_DIM (1..6) and SPX_UNIT_F (1, 2, 4, 8) defined, so the heavy
// instantiations compile in parallel.
#include "encode_dispatch.hpp"

#if !defined(SPX_UNIT_GRID) || !defined(SPX_UNIT_DIM) || !defined(SPX_UNIT_F)
#error "compile with -DSPX_UNIT_GRID=0|1 -DSPX_UNIT_DIM=1..6 -DSPX_UNIT_F=1|2|4|8"
#endif

namespace spx {
template <>
hipError_t encode_unit<(SPX_UNIT_GRID != 0), SPX_UNIT_DIM, SPX_UNIT_F>(const EncodeCall& c) {
    using Tag = std::conditional_t<SPX_UNIT_GRID != 0, GridTag, SimplexTag>;
    return dispatch_op<Tag, SPX_UNIT_DIM, SPX_UNIT_F>(c);
}
}  // namespace spx
