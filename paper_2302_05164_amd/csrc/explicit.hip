// Column kernels of the explicit step on uniform Lagrange boxes: dispatch to
// the instantiations (cells_q2_f64.hip, cells_q2_f32.hip, cells_q1.hip; the
// kernels themselves are in cells.h) and the face kernel that completes the
// nodes on column faces and segment ends.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "cellkit.h"

namespace pbf {

hipError_t launch_cells_q2_f64(int mode, const CellParams<double> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_cells_q2_f32(int mode, const CellParams<float> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_cells_q1_f64(int mode, const CellParams<double> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_cells_q1_f32(int mode, const CellParams<float> &p, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

namespace {
// Completion of the nodes on column faces and segment ends: fixed-order sum of
// the parity-slot partials of the (up to 8) columns/segments that contain them.
template <int MODE>
__global__ void __launch_bounds__(256) k_halo(const HaloParams h)
{
    FaceNode fn;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!face_node(t, h, fn)) return;
    const long long g = (long long)fn.gi + (long long)h.NX * fn.gj + (long long)h.NX * h.NY * fn.gk;
    const double f = face_sum(h.slots, h.GX + h.GY + h.GZ, t, fn);
    if (MODE == 0) {  // the slots hold T_n + dt f_0 / C~ and the other columns' increments
        h.Tout[g] = f;
    } else if (MODE == 2) {
        h.fout[g] = f;
    } else {
        h.fout[g] = f;
        h.Cout[g] = node_capacity(const_law(h.nlaw), h.Tin[g], int(fn.gi), int(fn.gj), int(fn.gk), h.P, h.NX,
                                  h.NY, h.NZ, h.hx, h.hy, h.hz);
    }
}

}  // namespace

namespace {
// Launch, with optional start/stop events recorded by the dispatch itself
// (kernel execution time only, no queue gaps).
template <typename K, typename A>
void launch_maybe_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                        const A &arg)
{
    if (e0) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, arg);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, arg);
}
}  // namespace

// 16 x 16 cells per column workgroup: measured fastest of 16x4, 16x8 and 16x16
// on 128x128x64 and 48x48x24 Q2 boxes (fewer column-face nodes, same per-lane work)
int column_height() { return 16; }

int resident_columns_per_cu(int ty) { return ty == 4 ? 8 : (ty == 8 ? 4 : 2); }

hipError_t launch_cells(int degree, int precision, int mode, int ty, const CellParams<double> &pd,
                        const CellParams<float> &pf, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (ty != 16) return hipErrorInvalidValue;  // columns of 16 x 16 cells (four waves)
    if (precision == PBF_PREC_FP64)
        return degree == 1 ? launch_cells_q1_f64(mode, pd, s, e0, e1) : launch_cells_q2_f64(mode, pd, s, e0, e1);
    if (mode == 2) return hipErrorInvalidValue;  // the Laplace reference runs in double precision
    return degree == 1 ? launch_cells_q1_f32(mode, pf, s, e0, e1) : launch_cells_q2_f32(mode, pf, s, e0, e1);
}

hipError_t launch_halo(int mode, const HaloParams &hp, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const long long n = hp.GX + hp.GY + hp.GZ;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (mode == 0) launch_maybe_timed(k_halo<0>, grid, block, s, e0, e1, hp);
    else if (mode == 1) launch_maybe_timed(k_halo<1>, grid, block, s, e0, e1, hp);
    else launch_maybe_timed(k_halo<2>, grid, block, s, e0, e1, hp);
    return hipGetLastError();
}

}  // namespace pbf
