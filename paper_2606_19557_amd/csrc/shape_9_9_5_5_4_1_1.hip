// Kernels of one descriptor shape (see nep_shapes.inc), both precisions.
#include "nep_pipeline.hpp"

NEP_SHAPE_TU(9, 9, 5, 5, 4, 1, 1)
