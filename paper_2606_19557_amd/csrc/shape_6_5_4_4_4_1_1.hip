// Kernels of one descriptor shape (see nep_shapes.inc), both precisions.
#include "nep_pipeline.hpp"

NEP_SHAPE_TU(6, 5, 4, 4, 4, 1, 1)
