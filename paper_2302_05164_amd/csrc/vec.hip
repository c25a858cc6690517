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
    if (h.dflag) return h.dflag[g] != 0;  // unstructured (octree) dof numbering
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

// out[c] = sum over blocks of partials[b*stride + c], c < ncomp: each thread
// adds a fixed strided subset in order, then a fixed tree (deterministic);
// MAXR: maximum instead of sum
template <bool MAXR>
__global__ void __launch_bounds__(kRedThreads) k_finish(const double *partials, int nblocks, int stride,
                                                        int ncomp, double *out)
{
    __shared__ double sh[kRedThreads];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
            const double v = partials[b * stride + c];
            s = MAXR ? fmax(s, v) : s + v;
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kRedThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                sh[threadIdx.x] = MAXR ? fmax(sh[threadIdx.x], sh[threadIdx.x + w]) : sh[threadIdx.x] + sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = sh[0];
        __syncthreads();
    }
}

// CG: r = -y (free) or 0, x = 0, z = r/diag, p = z; partials of r.z, r.r
__global__ void __launch_bounds__(kRedThreads) k_cg_start(const double *y, const double *diag, double *r,
                                                           double *z, double *p, double *x,
                                                           double *partials, const HaloParams h,
                                                           long long n)
{
    double s[2] = {0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double ri = node_dirichlet(i, h) ? 0.0 : -y[i];
        const double zi = ri / diag[i];
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        x[i] = 0.0;
        s[0] += ri * zi;
        s[1] += ri * ri;
    }
    block_sum<2>(s);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = s[1];
    }
}

__global__ void __launch_bounds__(kRedThreads) k_dot(const double *a, const double *b, double *partials,
                                                      long long n)
{
    double s[1] = {0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads)
        s[0] += a[i] * b[i];
    block_sum<1>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// alpha = rz/pAp; x += alpha p; r -= alpha Ap; z = r/diag; partials of r.z, r.r
__global__ void __launch_bounds__(kRedThreads) k_cg_update(double *x, double *r, double *z, const double *p,
                                                            const double *Ap, const double *diag,
                                                            double *partials, const double *scal,
                                                            int rz_old, long long n)
{
    const double alpha = scal[rz_old] / scal[CG_PAP];
    double s[2] = {0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * Ap[i];
        const double zi = ri / diag[i];
        r[i] = ri;
        z[i] = zi;
        s[0] += ri * zi;
        s[1] += ri * ri;
    }
    block_sum<2>(s);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = s[1];
    }
}

// beta = rz_new/rz_old; p = z + beta p
__global__ void k_cg_direction(double *p, const double *z, const double *scal, int rz_old, int rz_new,
                               long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = scal[rz_new] / scal[rz_old];
    p[i] = z[i] + beta * p[i];
}

// T^{i+1} = T^i + x on free nodes; partial maxima of |x| there
__global__ void __launch_bounds__(kRedThreads) k_picard_update(double *Ti, const double *x, double *partials,
                                                                const HaloParams h, long long n)
{
    double m = 0.0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        if (node_dirichlet(i, h)) continue;
        Ti[i] += x[i];
        m = fmax(m, fabs(x[i]));
    }
    __shared__ double sh[kRedThreads];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// energy terms over free nodes: C~ (T - T_prev), f_vol, -(f - f_vol)
__global__ void __launch_bounds__(kRedThreads) k_energy(const double *Tp, const double *T, const double *f,
                                                         const double *fv, const double *C, double *partials,
                                                         const HaloParams h, long long n)
{
    double s[3] = {0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        if (node_dirichlet(i, h)) continue;
        s[0] += C[i] * (T[i] - Tp[i]);
        s[1] += fv[i];
        s[2] -= f[i] - fv[i];
    }
    block_sum<3>(s);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) partials[3 * blockIdx.x + c] = s[c];
}

// number of non-finite entries and max |x| over the finite ones
__global__ void __launch_bounds__(kRedThreads) k_finite(const double *x, double *partials, long long n)
{
    double bad = 0.0, m = 0.0;
    for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kRedThreads) {
        const double v = x[i];
        if (isfinite(v)) m = fmax(m, fabs(v));
        else bad += 1.0;
    }
    double s[1] = {bad};
    block_sum<1>(s);
    __shared__ double sh[kRedThreads];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = sh[0];
    }
}

__global__ void k_sub(double *d, const double *a, const double *b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = a[i] - b[i];
}

__global__ void k_power_scale(double *v, const double *scal, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = v[i] / sqrt(scal[2]);
}

// ---- GMRES (restarted, classical Gram-Schmidt twice, Jacobi on the right) ----
constexpr int kMdotChunk = 16;  // Krylov vectors per multi-dot pass

// partials[b * kGmMax + i0 + i] = block b's part of w . V_{i0+i}, i < kc <= kMdotChunk
__global__ void __launch_bounds__(kRedThreads) k_mdot(const double *w, const double *V, long long ldv, int i0,
                                                       int kc, double *partials, long long n)
{
    double s[kMdotChunk];
#pragma unroll
    for (int i = 0; i < kMdotChunk; ++i) s[i] = 0.0;
    for (long long j = (long long)blockIdx.x * kRedThreads + threadIdx.x; j < n;
         j += (long long)gridDim.x * kRedThreads) {
        const double wj = w[j];
#pragma unroll
        for (int i = 0; i < kMdotChunk; ++i)
            if (i < kc) s[i] += wj * V[(long long)(i0 + i) * ldv + j];
    }
    block_sum<kMdotChunk>(s);
    if (threadIdx.x == 0)
        for (int i = 0; i < kc; ++i) partials[(long long)blockIdx.x * kGmMax + i0 + i] = s[i];
}

// w -= sum_{i<k} h_i V_i, the products subtracted in order of i
__global__ void k_maxpy(double *w, const double *V, long long ldv, int k, const double *h, long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double wj = w[j];
    for (int i = 0; i < k; ++i) wj -= h[i] * V[(long long)i * ldv + j];
    w[j] = wj;
}

// x += (sum_{i<k} y_i V_i) / diag
__global__ void k_gm_update(double *x, const double *V, long long ldv, int k, const double *y, const double *diag,
                            long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += y[i] * V[(long long)i * ldv + j];
    x[j] += s / diag[j];
}

__global__ void k_div(double *z, const double *v, const double *d, long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) z[j] = v[j] / d[j];
}

__global__ void k_div_scalar(double *v, const double *w, double h, long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) v[j] = w[j] / h;
}

__global__ void k_neg(double *b, const double *y, long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) b[j] = -y[j];
}

template <int P>
__global__ void k_layer_history(double *rc, long long stride, long long c0, long long c1, int cells_per_layer,
                                double hz, double Lz, double depth)
{
    constexpr int N = P + 1, NQ = N * N * N;
    const long long nc = c1 - c0;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * NQ) return;
    const int q = int(i / nc);
    const long long c = c0 + i % nc;
    const int qz = q / (N * N);
    constexpr double g0 = Tables<P>::gp(0), g1 = Tables<P>::gp(1), g2 = Tables<P>::gp(P);
    const double zeta = qz == 0 ? g0 : (qz == 1 ? g1 : g2);
    const double z = (double(c / cells_per_layer) + zeta) * hz;
    rc[(long long)q * stride + c] = (Lz - z <= depth) ? 0.0 : 1.0;
}

// ---- geometric multigrid on box lattices --------------------------------------
// A fine lattice of NXf = 2 NXc - 1 nodes per direction over the same box as
// the coarse lattice of NXc (the Q2 and Q1 node lattices of one mesh, or the Q1
// lattices of a mesh and its 2x coarsening).  Prolongation: trilinear
// interpolation (a fine node at an even index is a coarse node, at an odd
// index the average of its two coarse neighbours); restriction: its transpose.

// fine index i -> coarse indices and weights (1 or 2 of them)
__device__ __forceinline__ int mg_parents(int i, int &c0, int &c1)
{
    c0 = i >> 1;
    c1 = (i + 1) >> 1;
    return (i & 1) ? 2 : 1;
}

__global__ void k_mg_inject(double *c, const double *f, const HaloParams hc, int NXf, int NYf, long long n)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int I = int(g % hc.NX), J = int((g / hc.NX) % hc.NY), K = int(g / ((long long)hc.NX * hc.NY));
    c[g] = f[2LL * I + (long long)NXf * (2LL * J + (long long)NYf * 2LL * K)];
}

// c = P^T f, zero on the coarse Dirichlet rows
__global__ void k_mg_restrict(double *c, const double *f, const HaloParams hc, int NXf, int NYf, int NZf,
                              long long n)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    if (node_dirichlet(g, hc)) {
        c[g] = 0.0;
        return;
    }
    const int I = int(g % hc.NX), J = int((g / hc.NX) % hc.NY), K = int(g / ((long long)hc.NX * hc.NY));
    double s = 0.0;
    for (int dk = -1; dk <= 1; ++dk) {
        const int k = 2 * K + dk;
        if (k < 0 || k >= NZf) continue;
        const double wk = dk == 0 ? 1.0 : 0.5;
        for (int dj = -1; dj <= 1; ++dj) {
            const int j = 2 * J + dj;
            if (j < 0 || j >= NYf) continue;
            const double wj = dj == 0 ? 1.0 : 0.5;
            double row = 0.0;
            for (int di = -1; di <= 1; ++di) {
                const int i = 2 * I + di;
                if (i < 0 || i >= NXf) continue;
                row += (di == 0 ? 1.0 : 0.5) * f[i + (long long)NXf * (j + (long long)NYf * k)];
            }
            s += wk * wj * row;
        }
    }
    c[g] = s;
}

// f += P c on the free fine rows
__global__ void k_mg_prolong_add(double *f, const double *c, const HaloParams hf, int NXc, int NYc, long long n)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n || node_dirichlet(g, hf)) return;
    const int i = int(g % hf.NX), j = int((g / hf.NX) % hf.NY), k = int(g / ((long long)hf.NX * hf.NY));
    int i0, i1, j0, j1, k0, k1;
    const int ni = mg_parents(i, i0, i1), nj = mg_parents(j, j0, j1), nk = mg_parents(k, k0, k1);
    const double wi = ni == 2 ? 0.5 : 1.0, wj = nj == 2 ? 0.5 : 1.0, wk = nk == 2 ? 0.5 : 1.0;
    double s = 0.0;
    for (int b = 0; b < nk; ++b)
        for (int a = 0; a < nj; ++a)
            for (int e = 0; e < ni; ++e)
                s += c[(e ? i1 : i0) + (long long)NXc * ((a ? j1 : j0) + (long long)NYc * (b ? k1 : k0))];
    f[g] += wi * wj * wk * s;
}

// Chebyshev step of the smoother: d = c1 d + c2 r / diag, x = x + d (first step
// of a sweep from x = 0: d = c2 r / diag, x = d)
__global__ void k_cheb(double *x, double *d, const double *r, const double *diag, double c1, double c2, int from_zero,
                       long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double z = r[i] / diag[i];
    const double dn = c1 == 0.0 ? c2 * z : c1 * d[i] + c2 * z;
    d[i] = dn;
    x[i] = from_zero ? dn : x[i] + dn;
}

// a fixed pseudo-random vector in [-1, 1) (start of the eigenvalue estimates)
__global__ void k_seed(double *x, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ULL;
    h ^= h >> 29;
    x[i] = double(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Chebyshev step after an apply t = A x: d = c1 d + c2 (b - t) / diag, x += d
__global__ void k_cheb_res(double *x, double *d, const double *b, const double *t, const double *diag, double c1,
                           double c2, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double z = (b[i] - t[i]) / diag[i];
    const double dn = c1 == 0.0 ? c2 * z : c1 * d[i] + c2 * z;
    d[i] = dn;
    x[i] += dn;
}

// c = P^T (b - t), zero on the coarse Dirichlet rows
__global__ void k_mg_restrict_res(double *c, const double *b, const double *t, const HaloParams hc, int NXf, int NYf,
                                  int NZf, long long n)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    if (node_dirichlet(g, hc)) {
        c[g] = 0.0;
        return;
    }
    const int I = int(g % hc.NX), J = int((g / hc.NX) % hc.NY), K = int(g / ((long long)hc.NX * hc.NY));
    double s = 0.0;
    for (int dk = -1; dk <= 1; ++dk) {
        const int k = 2 * K + dk;
        if (k < 0 || k >= NZf) continue;
        const double wk = dk == 0 ? 1.0 : 0.5;
        for (int dj = -1; dj <= 1; ++dj) {
            const int j = 2 * J + dj;
            if (j < 0 || j >= NYf) continue;
            const double wj = dj == 0 ? 1.0 : 0.5;
            double row = 0.0;
            for (int di = -1; di <= 1; ++di) {
                const int i = 2 * I + di;
                if (i < 0 || i >= NXf) continue;
                const long long f = i + (long long)NXf * (j + (long long)NYf * k);
                row += (di == 0 ? 1.0 : 0.5) * (b[f] - t[f]);
            }
            s += wk * wj * row;
        }
    }
    c[g] = s;
}

__global__ void k_axpy(double *y, double a, const double *x, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_layer_history(int degree, double *rc, long long stride, long long c0, long long c1,
                                int cells_per_layer, double hz, double Lz, double depth, hipStream_t s)
{
    const long long n = (c1 - c0) * (degree + 1) * (degree + 1) * (degree + 1);
    if (n <= 0) return hipSuccess;
    if (degree == 1)
        hipLaunchKernelGGL(k_layer_history<1>, dim3(blocks_for(n, 256)), dim3(256), 0, s, rc, stride, c0, c1,
                           cells_per_layer, hz, Lz, depth);
    else
        hipLaunchKernelGGL(k_layer_history<2>, dim3(blocks_for(n, 256)), dim3(256), 0, s, rc, stride, c0, c1,
                           cells_per_layer, hz, Lz, depth);
    return hipGetLastError();
}

hipError_t launch_mdot(const double *w, const double *V, long long ldv, int k, double *partials, double *out,
                       long long n, hipStream_t s)
{
    for (int i0 = 0; i0 < k; i0 += kMdotChunk)
        hipLaunchKernelGGL(k_mdot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, w, V, ldv, i0,
                           k - i0 < kMdotChunk ? k - i0 : kMdotChunk, partials, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, kGmMax, k, out);
    return hipGetLastError();
}

hipError_t launch_maxpy(double *w, const double *V, long long ldv, int k, const double *h, long long n,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_maxpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, V, ldv, k, h, n);
    return hipGetLastError();
}

hipError_t launch_gm_update(double *x, const double *V, long long ldv, int k, const double *y, const double *diag,
                            long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_update, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, V, ldv, k, y, diag, n);
    return hipGetLastError();
}

hipError_t launch_div(double *z, const double *v, const double *d, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_div, dim3(blocks_for(n, 256)), dim3(256), 0, s, z, v, d, n);
    return hipGetLastError();
}

hipError_t launch_div_scalar(double *v, const double *w, double h, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_div_scalar, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, w, h, n);
    return hipGetLastError();
}

hipError_t launch_neg(double *b, const double *y, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_neg, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, y, n);
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 2, 2, scal);
    return hipGetLastError();
}

hipError_t launch_power_update(const double *f, const double *C, double *v, double *partials,
                               double *scal, const HaloParams &geom, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, f, C, v, partials,
                       geom, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 1, 1, scal + 2);
    return hipGetLastError();
}

hipError_t launch_power_scale(double *v, const double *scal, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_scale, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, scal, n);
    return hipGetLastError();
}

hipError_t launch_cg_start(const double *y, const double *diag, double *r, double *z, double *p,
                           double *x, double *partials, double *scal, const HaloParams &geom,
                           long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(kRedThreads), 0, s, y, diag, r, z, p, x,
                       partials, geom, n);
    // rz -> CG_RZ0, rr -> CG_RR; the initial rr is also kept as ||b||^2
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 2, 1,
                       scal + CG_RZ0);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials + 1, kRedBlocks, 2, 1,
                       scal + CG_RR);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials + 1, kRedBlocks, 2, 1,
                       scal + CG_BN2);
    return hipGetLastError();
}

hipError_t launch_cg_pap(const double *p, const double *Ap, double *partials, double *scal,
                         long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, p, Ap, partials, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 1, 1,
                       scal + CG_PAP);
    return hipGetLastError();
}

hipError_t launch_cg_update(double *x, double *r, double *z, const double *p, const double *Ap,
                            const double *diag, double *partials, double *scal, int rz_old,
                            long long n, hipStream_t s)
{
    const int rz_new = rz_old == CG_RZ0 ? CG_RZ1 : CG_RZ0;
    hipLaunchKernelGGL(k_cg_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, r, z, p, Ap, diag,
                       partials, scal, rz_old, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 2, 1,
                       scal + rz_new);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials + 1, kRedBlocks, 2, 1,
                       scal + CG_RR);
    return hipGetLastError();
}

hipError_t launch_cg_direction(double *p, const double *z, const double *scal, int rz_old, int rz_new,
                               long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_direction, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, z, scal, rz_old,
                       rz_new, n);
    return hipGetLastError();
}

hipError_t launch_picard_update(double *Ti, const double *x, double *partials, double *scal,
                                const HaloParams &geom, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_picard_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Ti, x, partials,
                       geom, n);
    hipLaunchKernelGGL(k_finish<true>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 1, 1,
                       scal + CG_DMAX);
    return hipGetLastError();
}

hipError_t launch_sub(double *d, const double *a, const double *b, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub, dim3(blocks_for(n, 256)), dim3(256), 0, s, d, a, b, n);
    return hipGetLastError();
}

hipError_t launch_energy(const double *Tp, const double *T, const double *f, const double *fv,
                         const double *C, double *partials, double *scal, const HaloParams &geom,
                         long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Tp, T, f, fv, C, partials, geom, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 3, 3,
                       scal + SC_ENERGY);
    return hipGetLastError();
}

hipError_t launch_finite(const double *x, double *partials, double *scal, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_finite, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, partials, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 2, 1,
                       scal + SC_FINITE);
    hipLaunchKernelGGL(k_finish<true>, dim3(1), dim3(kRedThreads), 0, s, partials + 1, kRedBlocks, 2, 1,
                       scal + SC_FINITE + 1);
    return hipGetLastError();
}


hipError_t launch_mg_inject(double *c, const double *f, const HaloParams &hc, int NXf, int NYf, hipStream_t s)
{
    const long long n = (long long)hc.NX * hc.NY * hc.NZ;
    hipLaunchKernelGGL(k_mg_inject, dim3(blocks_for(n, 256)), dim3(256), 0, s, c, f, hc, NXf, NYf, n);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(double *c, const double *f, const HaloParams &hc, int NXf, int NYf, int NZf,
                              hipStream_t s)
{
    const long long n = (long long)hc.NX * hc.NY * hc.NZ;
    hipLaunchKernelGGL(k_mg_restrict, dim3(blocks_for(n, 256)), dim3(256), 0, s, c, f, hc, NXf, NYf, NZf, n);
    return hipGetLastError();
}

hipError_t launch_mg_prolong_add(double *f, const double *c, const HaloParams &hf, int NXc, int NYc, hipStream_t s)
{
    const long long n = (long long)hf.NX * hf.NY * hf.NZ;
    hipLaunchKernelGGL(k_mg_prolong_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, f, c, hf, NXc, NYc, n);
    return hipGetLastError();
}

hipError_t launch_cheb(double *x, double *d, const double *r, const double *diag, double c1, double c2,
                       bool from_zero, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cheb, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, d, r, diag, c1, c2,
                       from_zero ? 1 : 0, n);
    return hipGetLastError();
}

hipError_t launch_cheb_res(double *x, double *d, const double *b, const double *t, const double *diag, double c1,
                           double c2, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cheb_res, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, d, b, t, diag, c1, c2, n);
    return hipGetLastError();
}

hipError_t launch_mg_restrict_res(double *c, const double *b, const double *t, const HaloParams &hc, int NXf, int NYf,
                                  int NZf, hipStream_t s)
{
    const long long n = (long long)hc.NX * hc.NY * hc.NZ;
    hipLaunchKernelGGL(k_mg_restrict_res, dim3(blocks_for(n, 256)), dim3(256), 0, s, c, b, t, hc, NXf, NYf, NZf, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double *y, double a, const double *x, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, y, a, x, n);
    return hipGetLastError();
}

hipError_t launch_seed(double *x, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_seed, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_dot_to(const double *a, const double *b, double *partials, double *out, long long n,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, partials, n);
    hipLaunchKernelGGL(k_finish<false>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 1, 1, out);
    return hipGetLastError();
}

}  // namespace pbf
