// Kernels of one descriptor shape (see nep_shapes.inc), both precisions.
#include "nep_pipeline.hpp"

NEP_SHAPE_TU(9, 9, 7, 5, 4, 0, 0)
