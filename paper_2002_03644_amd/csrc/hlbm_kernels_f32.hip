// FP32 instantiation of the HLBM kernels (deviation storage).
#define HLBM_REAL float
#define HLBM_NS f32
#include "hlbm_kernels_impl.hpp"
