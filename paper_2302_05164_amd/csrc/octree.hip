// Kernels of the operator on octree meshes with hanging nodes (gfx950).
//
// Same mathematics as on boxes (Section 4.2, eqs. diffusive_term_evaluation
// and vector_evaluation; Section 3.2, eq. forward_euler), with the gather G_e
// extended by the hanging-node constraints and per-leaf geometry (a leaf of
// level l is a box of size h0 / 2^l).
//
// Design (unstructured, two passes):
//  1. cell pass, one leaf per lane: gather the (p+1)^3 local values through the
//     per-cell index table (stored node-major, so lanes read consecutive
//     entries); a hanging local node reads its expanded constraint (rare, a
//     short CSR list); sum-factorized interpolation, law, source and
//     integration as on boxes; the element vector is written node-major to an
//     element buffer (coalesced);
//  2. node pass, one dof per lane: the transposed gather, sum over the dof's
//     (cell, local node, weight) entries in a fixed order (deterministic,
//     no atomics), then the lumped-capacity update, the assembled vectors,
//     or the Picard rows.
// Leaves are in Morton order and dofs numbered by first appearance, so both
// passes read neighbouring data from nearby addresses.
#include <hip/hip_runtime.h>

#include "cellkit.h"

namespace pbf {
namespace {

constexpr int kOctThreads = 128;

template <int P>
__device__ __forceinline__ void oct_gather(const OctDev &m, const double *T, int c, double *u)
{
    constexpr int NN = (P + 1) * (P + 1) * (P + 1);
    // all indices, then all regular values (loads in flight together; a hanging
    // node reads dof 0 and is replaced below), then the hanging nodes'
    // constraint sums, a pair of entries at a time (same summation order)
    int id[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) id[a] = m.cidx[(long long)a * m.n_cells + c];
#pragma unroll
    for (int a = 0; a < NN; ++a) u[a] = T[id[a] >= 0 ? id[a] : 0];
#pragma unroll
    for (int a = 0; a < NN; ++a) {
        if (id[a] >= 0) continue;
        const int h = -1 - id[a];
        const int j1 = m.hstart[h + 1];
        int j = m.hstart[h];
        double v = 0.0;
        for (; j + 2 <= j1; j += 2) {
            const double w0 = m.hw[j], w1 = m.hw[j + 1];
            const double t0 = T[m.hdof[j]], t1 = T[m.hdof[j + 1]];
            v = __builtin_fma(w0, t0, v);
            v = __builtin_fma(w1, t1, v);
        }
        if (j < j1) v = __builtin_fma(m.hw[j], T[m.hdof[j]], v);
        u[a] = v;
    }
}

struct CellGeo {
    double x0, y0, z0, hx, hy, hz, detJ, ih2x, ih2y, ih2z;
    bool top;  // the leaf touches the top face z = Lz
};

__device__ __forceinline__ CellGeo oct_geo(const OctDev &m, int c)
{
    CellGeo g;
    const int l = m.leaf[4 * c];
    const int si = 1 << (m.maxl - l);
    const double s = double(si);
    g.x0 = m.leaf[4 * c + 1] * m.ux;
    g.y0 = m.leaf[4 * c + 2] * m.uy;
    g.z0 = m.leaf[4 * c + 3] * m.uz;
    g.hx = s * m.ux;
    g.hy = s * m.uy;
    g.hz = s * m.uz;
    g.detJ = g.hx * g.hy * g.hz;
    g.ih2x = 1.0 / (g.hx * g.hx);
    g.ih2y = 1.0 / (g.hy * g.hy);
    g.ih2z = 1.0 / (g.hz * g.hz);
    g.top = m.leaf[4 * c + 3] + si == m.top_iz;
    return g;
}

// Gaussian surface flux of a top leaf onto its top node layer (fe += S^T q W)
template <int P>
__device__ __forceinline__ void surface_flux(const OctParams &p, const CellGeo &g, double sign, double *fe)
{
    using TB = Tables<P>;
    constexpr int N = P + 1;
    double qs[N * N];
    sfor<0, N * N>([&](auto ic) {
        constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
        constexpr double xi = TB::gp(i), et = TB::gp(j), w2 = TB::gw(i) * TB::gw(j);
        const double dxb = g.x0 + xi * g.hx - p.xb, dyb = g.y0 + et * g.hy - p.yb;
        qs[decltype(ic)::value] = w2 * g.hx * g.hy * p.src_amp *
                                  exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2);
    });
    sfor<0, N * N>([&](auto nc) {
        constexpr int ax = decltype(nc)::value % N, ay = decltype(nc)::value / N;
        double s = 0.0;
        sfor<0, N * N>([&](auto ic) {
            constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
            constexpr double cc = TB::S(i, ax) * TB::S(j, ay);
            if constexpr (cc != 0.0) s = __builtin_fma(cc, qs[decltype(ic)::value], s);
        });
        fe[(P * N + ay) * N + ax] += sign * s;
    });
}

// explicit step / assembly: element vectors of diffusion, source and surface flux
template <int P>
__global__ void __launch_bounds__(kOctThreads) __attribute__((amdgpu_waves_per_eu(P == 2 ? 1 : 2)))
k_oct_cells(const OctParams p)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    const int c = blockIdx.x * kOctThreads + threadIdx.x;
    if (c >= p.m.n_cells) return;
    ConstLaw<double> &law = const_law(p.law);
    const CellGeo g = oct_geo(p.m, c);
    double u[NN], t1[NN], t2[NN], v[NN], w[NN];
    oct_gather<P>(p.m, p.Tin, c, u);
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, v);
    const int hc = p.has_hist ? p.m.cell_hist[c] : -1;
    // hinge sums of all points, one hinge at a time (each coefficient read once;
    // every point adds its hinges in increasing order); hinges that no point of
    // the wave exceeds add exactly zero and are skipped
    double tmax = v[0];
#pragma unroll
    for (int a = 1; a < NN; ++a) tmax = fmax0(tmax, v[a]);
    int nh = 0;
    while (nh < law.n_hinge && __any(tmax > law.b[nh])) ++nh;
    double kq[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) kq[a] = law.k0;
    for (int i = 0; i < nh; ++i) {
        const double bi = law.b[i], dki = law.dk[i];
#pragma unroll
        for (int a = 0; a < NN; ++a) kq[a] = __builtin_fma(dki, fmax0(v[a] - bi, 0.0), kq[a]);
    }
    // the volume source's Gaussian once per (x, y) column of points
    const bool vol_src = p.laser_on && p.laser_kind == 1;
    double sq[N * N];
    if (vol_src) {
        sfor<0, N * N>([&](auto ic) {
            constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
            constexpr double xi = TB::gp(i), et = TB::gp(j);
            const double dxb = g.x0 + xi * g.hx - p.xb, dyb = g.y0 + et * g.hy - p.yb;
            sq[decltype(ic)::value] = p.src_amp * exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2);
        });
    }
#pragma unroll
    for (int a = 0; a < NN; ++a) w[a] = 0.0;
    // history of a z-plane of points, loaded together before the plane (the
    // updates would otherwise order each point's load behind the previous store)
    double rpl[N * N];
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
        if constexpr (qx == 0 && qy == 0) {
            if (hc >= 0) {
#pragma unroll
                for (int j = 0; j < N * N; ++j) rpl[j] = p.hist[(long long)(qz * N * N + j) * p.m.n_hist_cells + hc];
            }
        }
        auto gxf = [&](auto rc) { return v[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
        auto gyf = [&](auto rc) { return v[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
        auto gzf = [&](auto rc) { return v[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
        const double gx = rowdot<TagD<P>, qx, 0, N, false>(gxf, 0.0);
        const double gy = rowdot<TagD<P>, qy, 0, N, false>(gyf, 0.0);
        const double gz = rowdot<TagD<P>, qz, 0, N, false>(gzf, 0.0);
        const double T = v[q];
        const double kpl = kq[q];
        double k = kpl;
        if (hc >= 0) {  // consolidated fraction: r = max(r, g), updated before use
            const long long hi = (long long)q * p.m.n_hist_cells + hc;
            double r = rpl[qy * N + qx];
            const double gl = fmin0(fmax0((T - law.Ts) * law.inv_dT, 0.0), 1.0);
            if (gl > r) {
                r = gl;
                if (p.hist_write) p.hist[hi] = gl;
            }
            k = kpl * (r + law.phi * (1.0 - r));
        }
        constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
        const double kW = k * (wq * g.detJ);
        const double Fx = -kW * g.ih2x * gx, Fy = -kW * g.ih2y * gy, Fz = -kW * g.ih2z * gz;
        sfor<0, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
            if constexpr (dx != 0.0) w[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, w[tidx<N, 0>(r, qy, qz)]);
            if constexpr (dy != 0.0) w[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, w[tidx<N, 1>(r, qx, qz)]);
            if constexpr (dz != 0.0) w[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, w[tidx<N, 2>(r, qx, qy)]);
        });
        if (vol_src) {
            constexpr double ze = TB::gp(qz);
            const double depth = p.m.Lz - (g.z0 + ze * g.hz);
            if (depth >= 0.0 && depth <= p.h_powder) w[q] = __builtin_fma(wq * g.detJ, sq[qy * N + qx], w[q]);
        }
    });
    sweep<TagSt<P>, N, 0>(w, t1);
    sweep<TagSt<P>, N, 1>(t1, t2);
    sweep<TagSt<P>, N, 2>(t2, u);
    if (p.laser_on && p.laser_kind == 0 && g.top) surface_flux<P>(p, g, 1.0, u);
    if (p.re.on && g.top) {  // radiation and evaporation on the face z = Lz
        oct_gather<P>(p.m, p.Tin, c, t1);
        surface_loss_face<P>(p.re, g.hx, g.hy, [&](int ax, int ay) { return t1[(P * N + ay) * N + ax]; }, u);
    }
#pragma unroll
    for (int a = 0; a < NN; ++a) p.m.E[(long long)a * p.m.n_cells + c] = u[a];
}

// Picard operator C(Tc)/dt + K(Tk) with the history held fixed: MODE 0 the
// element vector of C x1 / dt + K x2 - f_vol, MODE 1 the element diagonal
template <int P, int MODE>
__global__ void __launch_bounds__(kOctThreads) __attribute__((amdgpu_waves_per_eu(P == 2 ? 1 : 2)))
k_oct_picard(const OctParams p)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    const int c = blockIdx.x * kOctThreads + threadIdx.x;
    if (c >= p.m.n_cells) return;
    ConstLaw<double> &law = const_law(p.law);
    const CellGeo g = oct_geo(p.m, c);
    const int hc = p.has_hist ? p.m.cell_hist[c] : -1;
    double u[NN], t1[NN], t2[NN], m[NN], kw[NN], fe[NN];
    oct_gather<P>(p.m, p.Tc, c, u);
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, m);
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr double wq = TB::gw(q % N) * TB::gw((q / N) % N) * TB::gw(q / (N * N));
        m[q] = wq * g.detJ * law.rho * law_c(law, m[q]) * p.inv_dt;
    });
    oct_gather<P>(p.m, p.Tk, c, u);
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, kw);
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr double wq = TB::gw(q % N) * TB::gw((q / N) % N) * TB::gw(q / (N * N));
        const double r = hc >= 0 ? p.hist[(long long)q * p.m.n_hist_cells + hc] : 1.0;
        kw[q] = wq * g.detJ * law_k(law, kw[q], r);
    });
    if constexpr (MODE == 0) {
        oct_gather<P>(p.m, p.x1, c, u);
        sweep<TagS<P>, N, 0>(u, t1);
        sweep<TagS<P>, N, 1>(t1, t2);
        sweep<TagS<P>, N, 2>(t2, u);
#pragma unroll
        for (int a = 0; a < NN; ++a) m[a] *= u[a];
        if (p.laser_on && p.laser_kind == 1) {
            sfor<0, NN>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
                constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
                constexpr double xi = TB::gp(qx), et = TB::gp(qy), ze = TB::gp(qz);
                const double depth = p.m.Lz - (g.z0 + ze * g.hz);
                if (depth >= 0.0 && depth <= p.h_powder) {
                    const double dxb = g.x0 + xi * g.hx - p.xb, dyb = g.y0 + et * g.hy - p.yb;
                    m[q] -= wq * g.detJ * p.src_amp * exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2);
                }
            });
        }
        oct_gather<P>(p.m, p.x2, c, u);
        sweep<TagS<P>, N, 0>(u, t1);
        sweep<TagS<P>, N, 1>(t1, t2);
        sweep<TagS<P>, N, 2>(t2, u);
        sfor<0, NN>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
            auto gxf = [&](auto rc) { return u[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
            auto gyf = [&](auto rc) { return u[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
            auto gzf = [&](auto rc) { return u[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
            const double Fx = kw[q] * g.ih2x * rowdot<TagD<P>, qx, 0, N, false>(gxf, 0.0);
            const double Fy = kw[q] * g.ih2y * rowdot<TagD<P>, qy, 0, N, false>(gyf, 0.0);
            const double Fz = kw[q] * g.ih2z * rowdot<TagD<P>, qz, 0, N, false>(gzf, 0.0);
            sfor<0, N>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
                if constexpr (dx != 0.0) m[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, m[tidx<N, 0>(r, qy, qz)]);
                if constexpr (dy != 0.0) m[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, m[tidx<N, 1>(r, qx, qz)]);
                if constexpr (dz != 0.0) m[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, m[tidx<N, 2>(r, qx, qy)]);
            });
        });
        integrate3<TagSt<P>, TagSt<P>, TagSt<P>, N>(m, fe);
        if (p.laser_on && p.laser_kind == 0 && g.top) surface_flux<P>(p, g, -1.0, fe);
    } else {
        double acc[NN];
        integrate3<TagS2t<P>, TagS2t<P>, TagS2t<P>, N>(m, fe);
        integrate3<TagDn2t<P>, TagS2t<P>, TagS2t<P>, N>(kw, acc);
#pragma unroll
        for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(g.ih2x, acc[a], fe[a]);
        integrate3<TagS2t<P>, TagDn2t<P>, TagS2t<P>, N>(kw, acc);
#pragma unroll
        for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(g.ih2y, acc[a], fe[a]);
        integrate3<TagS2t<P>, TagS2t<P>, TagDn2t<P>, N>(kw, acc);
#pragma unroll
        for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(g.ih2z, acc[a], fe[a]);
    }
#pragma unroll
    for (int a = 0; a < NN; ++a) p.m.E[(long long)a * p.m.n_cells + c] = fe[a];
}

// node pass (modes: see OctNodeParams)
template <int MODE>
__global__ void __launch_bounds__(256) k_oct_nodes(const OctNodeParams p)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p.m.n_dofs) return;
    // the dof's own values first, then its element entries four at a time (all
    // loads of a chunk in flight together; the sum keeps the entry order)
    const bool dir = p.m.dflag[i] != 0;
    const double T = MODE <= 1 ? p.Tin[i] : 0.0;
    const int e1 = p.m.nstart[i + 1];
    // weights in FP32 when the mesh's weights are exact there (uniform), else FP64
    auto gather = [&](auto wts) -> double {
        int e = p.m.nstart[i];
        double f = 0.0;
        for (; e + 4 <= e1; e += 4) {
            double w[4], v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = double(wts[e + j]);
                v[j] = p.m.E[p.m.nslot[e + j]];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) f = __builtin_fma(MODE == 3 ? w[j] * w[j] : w[j], v[j], f);
        }
        for (; e < e1; ++e) {
            const double w = double(wts[e]);
            f = __builtin_fma(MODE == 3 ? w * w : w, p.m.E[p.m.nslot[e]], f);
        }
        return f;
    };
    const double f = p.m.nw_f32 ? gather(p.m.nwf) : gather(p.m.nw);
    if constexpr (MODE <= 1) {
        ConstLaw<double> &L = const_law(p.nlaw);
        const double C = L.rho * law_c(L, T) * p.m.mass[i];
        if constexpr (MODE == 0) {
            p.Tout[i] = dir ? p.T_D : T + p.dt * f / C;
        } else {
            p.fout[i] = f;
            p.Cout[i] = C;
        }
    } else if constexpr (MODE == 2) {
        p.Tout[i] = dir ? 0.0 : f;
    } else {
        p.Tout[i] = dir ? 1.0 : f;
    }
}

// initial consolidated fraction: 0 at Gauss points at most powder_depth below
// the top face, 1 elsewhere (point-major history of the history leaves)
template <int P>
__global__ void k_oct_init_history(const OctDev m, double depth, double *rc)
{
    constexpr int N = P + 1, NQ = N * N * N;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)m.n_hist_cells * NQ) return;
    const int q = int(i / m.n_hist_cells), hc = int(i % m.n_hist_cells);
    constexpr double g0 = Tables<P>::gp(0), g1 = Tables<P>::gp(1), g2 = Tables<P>::gp(P);
    const int qz = q / (N * N);
    const double zeta = qz == 0 ? g0 : (qz == 1 ? g1 : g2);
    const double z = m.hist_z[2 * hc] + zeta * m.hist_z[2 * hc + 1];
    rc[i] = (m.Lz - z <= depth) ? 0.0 : 1.0;
}

// remesh: the old finite element field at the new dofs (cell < 0: a dof above
// the old top of a growing build, which starts at T0); history copied, reset,
// or (coarsened parents of a growing build) the minimum over a group of old points
template <int P>
__global__ void k_oct_transfer_T(const OctDev old, const double *T_old, const int32_t *cell, const double *xi,
                                 long long n, double *T_new, double T0)
{
    constexpr int N = P + 1, NN = N * N * N;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (cell[i] < 0) {
        T_new[i] = T0;
        return;
    }
    double u[NN];
    oct_gather<P>(old, T_old, cell[i], u);
    const double x = xi[3 * i], y = xi[3 * i + 1], z = xi[3 * i + 2];
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < NN; ++a)
        v = __builtin_fma(lagrange1(P, a % N, x) * lagrange1(P, (a / N) % N, y) * lagrange1(P, a / (N * N), z),
                          u[a], v);
    T_new[i] = v;
}

__global__ void k_oct_transfer_hist(const double *rc_old, const int32_t *src, long long n, const int32_t *grp_start,
                                    const int32_t *grp_idx, double *rc_new)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int s = src[i];
    if (s >= -2) {
        rc_new[i] = s >= 0 ? rc_old[s] : (s == -1 ? 0.0 : 1.0);
        return;
    }
    const int g = -3 - s;
    double m = rc_old[grp_idx[grp_start[g]]];
    for (int j = grp_start[g] + 1; j < grp_start[g + 1]; ++j) m = fmin(m, rc_old[grp_idx[j]]);
    rc_new[i] = m;
}

inline unsigned nblocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_oct_cells(int degree, const OctParams &p, hipStream_t s)
{
    const dim3 g(nblocks(p.m.n_cells, kOctThreads)), b(kOctThreads);
    if (degree == 1) hipLaunchKernelGGL(k_oct_cells<1>, g, b, 0, s, p);
    else hipLaunchKernelGGL(k_oct_cells<2>, g, b, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_oct_picard(int degree, int mode, const OctParams &p, hipStream_t s)
{
    const dim3 g(nblocks(p.m.n_cells, kOctThreads)), b(kOctThreads);
    if (degree == 1) {
        if (mode == 0) hipLaunchKernelGGL((k_oct_picard<1, 0>), g, b, 0, s, p);
        else hipLaunchKernelGGL((k_oct_picard<1, 1>), g, b, 0, s, p);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_oct_picard<2, 0>), g, b, 0, s, p);
        else hipLaunchKernelGGL((k_oct_picard<2, 1>), g, b, 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_oct_nodes(int mode, const OctNodeParams &p, hipStream_t s)
{
    const dim3 g(nblocks(p.m.n_dofs, 256)), b(256);
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_oct_nodes<0>, g, b, 0, s, p); break;
    case 1: hipLaunchKernelGGL(k_oct_nodes<1>, g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL(k_oct_nodes<2>, g, b, 0, s, p); break;
    default: hipLaunchKernelGGL(k_oct_nodes<3>, g, b, 0, s, p); break;
    }
    return hipGetLastError();
}

hipError_t launch_oct_init_history(const OctDev &m, int degree, double powder_depth, double *rc, hipStream_t s)
{
    const long long n = (long long)m.n_hist_cells * (degree + 1) * (degree + 1) * (degree + 1);
    if (n == 0) return hipSuccess;
    if (degree == 1) hipLaunchKernelGGL(k_oct_init_history<1>, dim3(nblocks(n, 256)), dim3(256), 0, s, m, powder_depth, rc);
    else hipLaunchKernelGGL(k_oct_init_history<2>, dim3(nblocks(n, 256)), dim3(256), 0, s, m, powder_depth, rc);
    return hipGetLastError();
}

hipError_t launch_oct_transfer(int degree, const OctDev &old, const double *T_old, const int32_t *cell,
                               const double *xi, int64_t n, double *T_new, double T0, const double *rc_old,
                               const int32_t *src, int64_t n_hist, const int32_t *grp_start, const int32_t *grp_idx,
                               double *rc_new, hipStream_t s)
{
    if (n > 0) {
        if (degree == 1)
            hipLaunchKernelGGL(k_oct_transfer_T<1>, dim3(nblocks(n, 256)), dim3(256), 0, s, old, T_old, cell, xi,
                               (long long)n, T_new, T0);
        else
            hipLaunchKernelGGL(k_oct_transfer_T<2>, dim3(nblocks(n, 256)), dim3(256), 0, s, old, T_old, cell, xi,
                               (long long)n, T_new, T0);
    }
    if (n_hist > 0)
        hipLaunchKernelGGL(k_oct_transfer_hist, dim3(nblocks(n_hist, 256)), dim3(256), 0, s, rc_old, src,
                           (long long)n_hist, grp_start, grp_idx, rc_new);
    return hipGetLastError();
}

}  // namespace pbf
