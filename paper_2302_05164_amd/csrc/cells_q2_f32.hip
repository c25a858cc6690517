// Instantiations of the column kernels of cells.h: Q2 cells with the FP32 operator
// (one translation unit each, so that they compile in parallel).
#include "cells.h"

namespace pbf {
hipError_t launch_cells_q2_f32(int mode, const CellParams<float> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (mode == 0) return launch_cells_inst<2, float, 0>(p, s, e0, e1);
    return launch_cells_inst<2, float, 1>(p, s, e0, e1);
}
}  // namespace pbf
