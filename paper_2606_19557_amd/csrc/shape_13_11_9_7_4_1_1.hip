// Kernels of one descriptor shape (see nep_shapes.inc), both precisions.
#include "nep_pipeline.hpp"

NEP_SHAPE_TU(13, 11, 9, 7, 4, 1, 1)
