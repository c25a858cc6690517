// Vector kernels of the pbftherm library: state initialization and the
// power iteration of the explicit stability estimate (Section 3.2,
// eq. explicit_time_step).  Reductions are deterministic: each block writes a
// partial sum in a fixed tree order and one block adds the partials in index
// order.
#include <hip/hip_runtime.h>

#include "pbf_internal.h"

namespace pbf {
namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ bool node_dirichlet(long long g, const HaloParams &h)
{
    const long long NXY = (long long)h.NX * h.NY;
    const int i = int(g % h.NX), j = int((g / h.NX) % h.NY), k = int(g / NXY);
    const unsigned m = h.dmask;
    return ((m & 1u) && i == 0) || ((m & 2u) && i == h.NX - 1) || ((m & 4u) && j == 0) ||
           ((m & 8u) && j == h.NY - 1) || ((m & 16u) && k == 0) || ((m & 32u) && k == h.NZ - 1);
}

// block-wide sum of NV values; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][kRedThreads];
    for (int c = 0; c < NV; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < NV; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        __syncthreads();
    }
    for (int c = 0; c < NV; ++c) v[c] = sh[c][0];
}

__global__ void k_fill(double *x, double v, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_set_dirichlet(double *T, const HaloParams h, double T_D, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && node_dirichlet(i, h)) T[i] = T_D;
}

struct HistInit {
    int n_hist_cells, nq1, hist_layers, cells_per_layer;
    unsigned char powder[96];  // [layer][qz]: 1 if the Gauss level starts as powder
};

__global__ void k_init_history(double *rc, const HistInit hi)
{
    const long long n = (long long)hi.n_hist_cells * hi.nq1 * hi.nq1 * hi.nq1;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q = int(i / hi.n_hist_cells);
    const long long c = i % hi.n_hist_cells;
    const int qz = q / (hi.nq1 * hi.nq1);
    const int layer = int(c / hi.cells_per_layer);
    rc[i] = hi.powder[layer * hi.nq1 + qz] ? 0.0 : 1.0;
}

// partial sums of  sum_free (-f v)  and  sum_free C v^2
__global__ void __launch_bounds__(kRedThreads) k_power_dots(const double *f, const double *C,
                                                             const double *v, double *partials,
                                                             const HaloParams h, long long n)
{
    double s[2] = {0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        if (node_dirichlet(i, h)) continue;
        s[0] += -f[i] * v[i];
        s[1] += C[i] * v[i] * v[i];
    }
    block_sum<2>(s);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = s[1];
    }
}

// v <- -f/C on free nodes (0 on Dirichlet nodes); partial sums of v^2
__global__ void __launch_bounds__(kRedThreads) k_power_update(const double *f, const double *C,
                                                               double *v, double *partials,
                                                               const HaloParams h, long long n)
{
    double s[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double x = node_dirichlet(i, h) ? 0.0 : -f[i] / C[i];
        v[i] = x;
        s[0] += x * x;
    }
    block_sum<1>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// out[c] = sum over blocks of partials[b*nv + c], in block order
__global__ void k_finish(const double *partials, int nblocks, int nv, double *out)
{
    const int c = threadIdx.x;
    if (c >= nv) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partials[b * nv + c];
    out[c] = s;
}

__global__ void k_power_scale(double *v, const double *scal, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = v[i] / sqrt(scal[2]);
}

inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_fill(double *x, double v, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}

hipError_t launch_init_dirichlet(double *T, const HaloParams &geom, double T_D, hipStream_t s)
{
    const long long n = (long long)geom.NX * geom.NY * geom.NZ;
    hipLaunchKernelGGL(k_set_dirichlet, dim3(blocks_for(n, 256)), dim3(256), 0, s, T, geom, T_D, n);
    return hipGetLastError();
}

hipError_t launch_init_history(double *rc, int n_hist_cells, int nq1, const int *qz_powder_mask,
                               int hist_layers, int nx, int ny, hipStream_t s)
{
    HistInit hi{};
    hi.n_hist_cells = n_hist_cells;
    hi.nq1 = nq1;
    hi.hist_layers = hist_layers;
    hi.cells_per_layer = nx * ny;
    if (hist_layers * nq1 > 96) return hipErrorInvalidValue;
    for (int i = 0; i < hist_layers * nq1; ++i) hi.powder[i] = (unsigned char)(qz_powder_mask[i] != 0);
    const long long n = (long long)n_hist_cells * nq1 * nq1 * nq1;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_history, dim3(blocks_for(n, 256)), dim3(256), 0, s, rc, hi);
    return hipGetLastError();
}

hipError_t launch_power_dots(const double *f, const double *C, const double *v, double *partials,
                             double *scal, const HaloParams &geom, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_dots, dim3(kRedBlocks), dim3(kRedThreads), 0, s, f, C, v, partials,
                       geom, n);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, partials, kRedBlocks, 2, scal);
    return hipGetLastError();
}

hipError_t launch_power_update(const double *f, const double *C, double *v, double *partials,
                               double *scal, const HaloParams &geom, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, f, C, v, partials,
                       geom, n);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, partials, kRedBlocks, 1, scal + 2);
    return hipGetLastError();
}

hipError_t launch_power_scale(double *v, const double *scal, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_scale, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, scal, n);
    return hipGetLastError();
}

}  // namespace pbf
