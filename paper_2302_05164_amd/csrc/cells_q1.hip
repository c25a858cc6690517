// Instantiations of the column kernels of cells.h: Q1 cells (double precision and the FP32 operator)
// (one translation unit each, so that they compile in parallel).
#include "cells.h"

namespace pbf {
hipError_t launch_cells_q1_f64(int mode, const CellParams<double> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (mode == 0) return launch_cells_inst<1, double, 0>(p, s, e0, e1);
    if (mode == 1) return launch_cells_inst<1, double, 1>(p, s, e0, e1);
    return launch_cells_inst<1, double, 2>(p, s, e0, e1);
}

hipError_t launch_cells_q1_f32(int mode, const CellParams<float> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (mode == 0) return launch_cells_inst<1, float, 0>(p, s, e0, e1);
    return launch_cells_inst<1, float, 1>(p, s, e0, e1);
}
}  // namespace pbf
