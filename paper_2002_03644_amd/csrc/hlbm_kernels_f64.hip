// FP64 instantiation of the HLBM kernels (absolute storage); compiled
// without floating-point contraction.
#define HLBM_REAL double
#define HLBM_NS f64
// tile shapes of the batched tile kernel that keep two waves per SIMD in FP64
#define HLBM_TILE_SHAPES(X) X(32, 8, 256) X(32, 16, 256) X(64, 8, 256)
#define HLBM_TILE2_SHAPES(X)
#include "hlbm_kernels_impl.hpp"
