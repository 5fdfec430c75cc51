// Instantiations of the FP32 cross-correlation kernel for tile_size_x = 8.
#include "xcorr_f32.hpp"
GT_XCORR_TABLE(8)
