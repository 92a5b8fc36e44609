// FP64 instantiation of the HLBM kernels (absolute storage); compiled
// without floating-point contraction.
#define HLBM_REAL double
#define HLBM_NS f64
#include "hlbm_kernels_impl.hpp"
