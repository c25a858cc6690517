// Cell-batched sum-factorization kernels of the nonlinear heat operator on
// uniform Lagrange boxes (gfx950).
//
// What is computed (Section 4.2, eqs. diffusive_term_evaluation and
// vector_evaluation; Section 3.2, eq. forward_euler):
//   f = sum_e G_e^T [ S_grad^T D_e S_grad + S_val^T q_vol ] G_e T,
//   T_{n+1} = T_n + dt f / C~ at free nodes, T_D at Dirichlet nodes,
// with the material law of Section 2 evaluated at every quadrature point and
// the lumped capacity C~_i = rho c(T_i) M~_i (row-sum lumped mass, positive for
// Q1 and Q2) evaluated at the node when it is updated.
//
// Design (one workgroup = a column of 16x16 cells, one cell per lane, marching
// up through a segment of cell layers):
//  1. per layer, the node planes of the layer are staged in LDS with coalesced
//     row loads and each lane gathers its cell;
//  2. each lane interpolates to the Gauss points with three 1D sweeps in
//     registers (compile-time 1D tables, structural zeros and ones removed),
//     differentiates by Gauss-point collocation, evaluates the material law and
//     the laser source, and integrates back with the transposed sweeps;
//  3. cell vectors go to a conflict-free LDS staging array; every node then
//     adds the contributions of its (at most 4) cells of the layer in a fixed
//     order, so results are bitwise reproducible;
//  4. the top node plane of a layer is carried in LDS to the next layer, whose
//     bottom plane it is; nodes that are then complete get the lumped-mass
//     update right away and T_{n+1} is written once (the GPU counterpart of
//     interleaving cell loop and vector update, Section 4.2.2);
//  5. nodes on the side faces of a column or on the end planes of a segment
//     store their partial sums in one of 8 slot arrays chosen by the parity of
//     the column and segment coordinates (neighbours sharing a node differ in
//     parity); a second kernel adds the <= 8 partials in a fixed order and
//     applies the update.
// Workgroups are mapped so that each XCD gets a contiguous range of columns
// and segments (neighbours then share face nodes in the same L2).
#include <hip/hip_runtime.h>

#include "pbf_internal.h"

namespace pbf {
namespace {

template <typename R> __device__ __forceinline__ R ffma(R a, R b, R c);
template <> __device__ __forceinline__ double ffma<double>(double a, double b, double c)
{
    return __builtin_fma(a, b, c);
}
template <> __device__ __forceinline__ float ffma<float>(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}
// The material law is read through the constant address space: the loads are
// scalar, cached in the scalar cache and known not to alias the history stores.
template <typename R>
using ConstLaw = const __attribute__((address_space(4))) Law<R>;
template <typename R>
__device__ __forceinline__ ConstLaw<R> &const_law(const Law<R> *p)
{
    return *(ConstLaw<R> *)p;
}

// Kernel parameters re-read inside the layer loop through a laundered pointer
// to the kernel-argument segment (scalar loads near their uses) instead of
// being held in scalar registers across the whole loop.
template <typename T>
using AS4 = const __attribute__((address_space(4))) T;
template <typename T>
__device__ __forceinline__ AS4<T> *kernarg_params()
{
    AS4<T> *kp = (AS4<T> *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(kp));
    return kp;
}

template <typename R> __device__ __forceinline__ R fmax0(R a, R b) { return a > b ? a : b; }
template <typename R> __device__ __forceinline__ R fmin0(R a, R b) { return a < b ? a : b; }

// compile-time loop
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// acc + sum_i M(row, i) x(i), terms with an exactly zero coefficient dropped and
// unit coefficients added without a multiply.
template <class M, int row, int i, int N, bool started, typename R, typename X>
__device__ __forceinline__ R rowdot(const X &x, R acc)
{
    if constexpr (i == N) {
        if constexpr (started) return acc;
        else return R(0);
    } else {
        constexpr double c = M::c(row, i);
        if constexpr (c == 0.0) {
            return rowdot<M, row, i + 1, N, started>(x, acc);
        } else {
            R xi = x(std::integral_constant<int, i>{});
            R nacc;
            if constexpr (!started) nacc = (c == 1.0) ? xi : R(c) * xi;
            else nacc = (c == 1.0) ? acc + xi : ffma(R(c), xi, acc);
            return rowdot<M, row, i + 1, N, true>(x, nacc);
        }
    }
}

// flat index of a (z,y,x) register tensor with extent N per direction; `a` runs
// along direction DIM, (i, j) along the other two in increasing order
template <int N, int DIM>
__device__ constexpr int tidx(int a, int i, int j)
{
    if constexpr (DIM == 0) return (j * N + i) * N + a;
    else if constexpr (DIM == 1) return (j * N + a) * N + i;
    else return (a * N + j) * N + i;
}

// out = M applied along DIM (every line of the tensor)
template <class M, int N, int DIM, typename R>
__device__ __forceinline__ void sweep(const R *in, R *out)
{
    sfor<0, N>([&](auto ic) {
        sfor<0, N>([&](auto jc) {
            constexpr int I = decltype(ic)::value, J = decltype(jc)::value;
            auto get = [&](auto ac) {
                constexpr int A = decltype(ac)::value;
                return in[tidx<N, DIM>(A, I, J)];
            };
            sfor<0, N>([&](auto oc) {
                constexpr int O = decltype(oc)::value;
                out[tidx<N, DIM>(O, I, J)] = rowdot<M, O, 0, N, false>(get, R(0));
            });
        });
    });
}

// Flux and source at the Gauss points of one cell, accumulated into the
// collocation-space integrand w.  FAST: at most one hinge of the law active, no
// history and no source in the wave (uniform branch-free straight-line code).
template <int P, typename R, bool FAST, typename PP, typename L>
__device__ __forceinline__ void flux_points(PP &p, L &law, const R *v, R *w, int nhinge, bool melt,
                                            bool has_hist, long long hc, bool src_cell, int cx, int cy,
                                            int cz)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    const R k0 = law.k0;
    const R b0 = law.b[0];
    const R dk0 = nhinge > 0 ? R(law.dk[0]) : R(0);
    const R detJ = p.detJ, ih2x = p.ih2x, ih2y = p.ih2y, ih2z = p.ih2z;
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
        // reference gradient by Gauss-point collocation
        auto gxf = [&](auto rc) { return v[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
        auto gyf = [&](auto rc) { return v[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
        auto gzf = [&](auto rc) { return v[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
        const R gx = rowdot<TagD<P>, qx, 0, N, false>(gxf, R(0));
        const R gy = rowdot<TagD<P>, qy, 0, N, false>(gyf, R(0));
        const R gz = rowdot<TagD<P>, qz, 0, N, false>(gzf, R(0));
        const R T = v[q];
        // conductivity (Section 2): hinge sum truncated to the breakpoints
        // that some lane of the wave exceeds
        R k;
        if constexpr (FAST) {
            k = ffma(dk0, fmax0(T - b0, R(0)), k0);
        } else {
            R kpl = k0;
            for (int i = 0; i < nhinge; ++i) kpl = ffma(law.dk[i], fmax0(T - law.b[i], R(0)), kpl);
            k = kpl;
            if (has_hist) {
                const long long hi = (long long)q * p.n_hist_cells + hc;
                R r = R(p.hist[hi]);
                if (melt) {
                    const R g = fmin0(fmax0((T - law.Ts) * law.inv_dT, R(0)), R(1));
                    if (g > r) {  // r_c = max(r_c, g): update before use
                        r = g;
                        p.hist[hi] = double(g);
                    }
                }
                // k = (1-r) k_p + g k_m + (r-g) k_s with k_m = k_s = k(T), k_p = phi k(T)
                k = kpl * (r + law.phi * (R(1) - r));
            }
        }
        constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
        const R kW = k * (R(wq) * detJ);
        // flux -k W J^{-1} J^{-T} grad T, collocation transpose
        const R Fx = -kW * ih2x * gx, Fy = -kW * ih2y * gy, Fz = -kW * ih2z * gz;
        sfor<0, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
            if constexpr (dx != 0.0) w[tidx<N, 0>(r, qy, qz)] = ffma(R(dx), Fx, w[tidx<N, 0>(r, qy, qz)]);
            if constexpr (dy != 0.0) w[tidx<N, 1>(r, qx, qz)] = ffma(R(dy), Fy, w[tidx<N, 1>(r, qx, qz)]);
            if constexpr (dz != 0.0) w[tidx<N, 2>(r, qx, qy)] = ffma(R(dz), Fz, w[tidx<N, 2>(r, qx, qy)]);
        });
        if constexpr (!FAST) {
            if (src_cell) {
                constexpr double xiq = TB::gp(qx), etq = TB::gp(qy), zeq = TB::gp(qz);
                const double zq = (cz + zeq) * p.hz;
                const double depth = p.Lz - zq;
                if (depth >= 0.0 && depth <= p.h_powder) {
                    const double dxb = (cx + xiq) * p.hx - p.xb;
                    const double dyb = (cy + etq) * p.hy - p.yb;
                    const double s = p.src_amp * exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2);
                    w[q] = ffma(R(wq) * detJ, R(s), w[q]);
                }
            }
        }
    });
}

// ---------------------------------------------------------------------------
// one cell: nodal values u -> element vector fe (diffusion, source, surface
// flux).  Values are relative to Tref (zero in double precision).
// ---------------------------------------------------------------------------
template <int P, typename R, typename PP>
__device__ __forceinline__ void cell_operator(PP &p, const Law<R> *lawp, const R *u, int cx, int cy,
                                              int cz, R *fe)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    R t1[NN], t2[NN], v[NN];
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, v);  // values at the Gauss points

    // Wave-uniform truncation of the material law: hinge i (slope change at
    // breakpoint b_i) contributes only where T > b_i, and the latent heat and
    // history only where T >= T_s.  Terms that no Gauss point of the wave
    // reaches are exactly zero and are skipped (called by active lanes only).
    ConstLaw<R> &law = const_law(lawp);
    R tmax = v[0];
#pragma unroll
    for (int q = 1; q < NN; ++q) tmax = fmax0(tmax, v[q]);
    int nhinge = 0;
    while (nhinge < law.n_hinge && __any(tmax > law.b[nhinge])) ++nhinge;
    const bool melt = __any(tmax >= law.Ts);  // history changes only from T_s up

    // history of powder cells (point-major storage)
    const bool has_hist = cz >= p.hist_cz0;
    const long long hc = has_hist ? (long long)cx + (long long)p.nx * (cy + (long long)p.ny * (cz - p.hist_cz0)) : 0;
    const bool src_cell = p.laser_on && p.laser_kind == 1 && cz >= p.src_cz0;

    R w[NN];  // collocation-space integrand of f
#pragma unroll
    for (int q = 0; q < NN; ++q) w[q] = R(0);
    // Most cells of a scan are cold, consolidated and away from the beam: for
    // them the 27 points run as one straight-line block (one hinge at most, no
    // history, no source), which lets the scheduler interleave independent
    // points.  Both paths evaluate the same arithmetic.
    if (nhinge <= 1 && !has_hist && !src_cell)
        flux_points<P, R, true>(p, law, v, w, nhinge, melt, false, 0, false, cx, cy, cz);
    else
        flux_points<P, R, false>(p, law, v, w, nhinge, melt, has_hist, hc, src_cell, cx, cy, cz);

    // integrate f: transposed interpolation sweeps
    sweep<TagSt<P>, N, 0>(w, t1);
    sweep<TagSt<P>, N, 1>(t1, t2);
    sweep<TagSt<P>, N, 2>(t2, fe);

    // Gaussian surface flux on the top face (Neumann input, z = Lz)
    if (p.laser_on && p.laser_kind == 0 && cz == p.nz - 1) {
        R qs[N * N];
        sfor<0, N * N>([&](auto ic) {
            constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
            constexpr double xi = TB::gp(i), et = TB::gp(j);
            const double dxb = (cx + xi) * p.hx - p.xb;
            const double dyb = (cy + et) * p.hy - p.yb;
            constexpr double w2 = TB::gw(i) * TB::gw(j);
            qs[decltype(ic)::value] =
                R(w2 * p.hx * p.hy * p.src_amp * exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2));
        });
        // 2D transposed interpolation onto the top node layer
        sfor<0, N>([&](auto ac) {
            constexpr int ax = decltype(ac)::value;
            sfor<0, N>([&](auto bc) {
                constexpr int ay = decltype(bc)::value;
                R s = R(0);
                sfor<0, N * N>([&](auto ic) {
                    constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
                    constexpr double c = TB::S(i, ax) * TB::S(j, ay);
                    if constexpr (c != 0.0) s = ffma(R(c), qs[decltype(ic)::value], s);
                });
                fe[(P * N + ay) * N + ax] += s;
            });
        });
    }
}

__device__ __forceinline__ bool on_dirichlet(unsigned m, int i, int j, int k, int NX, int NY, int NZ)
{
    return ((m & 1u) && i == 0) || ((m & 2u) && i == NX - 1) || ((m & 4u) && j == 0) ||
           ((m & 8u) && j == NY - 1) || ((m & 16u) && k == 0) || ((m & 32u) && k == NZ - 1);
}

__device__ __forceinline__ bool is_face(int g, int S, int n)  // interior tile face
{
    return g > 0 && g < n - 1 && (g % S) == 0;
}

// lumped capacity C~_i = rho c(T_i) M~_i at node (i,j,k), in double precision;
// hinges of the law that no active lane of the wave exceeds are skipped
__device__ __forceinline__ double node_capacity(ConstLaw<double> &L, double T, int i, int j, int k,
                                                int P, int NX, int NY, int NZ, double hx, double hy,
                                                double hz)
{
    double c = L.c0;
    if (L.n_hinge > 0 && __any(T > L.b[0])) {
        if (L.n_hinge > 1 && __any(T > L.b[1])) {
            int nh = 2;
            while (nh < L.n_hinge && __any(T > L.b[nh])) ++nh;
            for (int h = 0; h < nh; ++h) c = __builtin_fma(L.dc[h], fmax0(T - L.b[h], 0.0), c);
        } else {
            c = __builtin_fma(L.dc[0], fmax0(T - L.b[0], 0.0), c);
        }
    }
    if (T >= L.Ts && T <= L.Tl) c += L.lat;
    const double m = lumped_mass_1d(i, NX, P, hx) * lumped_mass_1d(j, NY, P, hy) *
                     lumped_mass_1d(k, NZ, P, hz);
    return L.rho * c * m;
}

// MODE 0: explicit step (fused update into Tout); MODE 1: assemble f and C~.
//
// Node ownership inside a column: the lane of cell (lx, ly) owns the nodes of
// its cell with local x and y indices in 1..P (plus index 0 on the column's
// low faces).  Own contributions come straight from registers; the shared
// contributions of the right, upper and diagonal neighbour cells come from a
// small LDS staging area (each cell stages its x = 0 plane and its y = 0 row);
// the top node plane is carried per lane to the next layer.  The sum order of
// every node is fixed: carry, own, right, upper, diagonal.
template <int P, typename R, int MODE, int kTY>
__global__ void __launch_bounds__(kTX * kTY) __attribute__((amdgpu_waves_per_eu(P == 2 && sizeof(R) == 8 ? 2 : (P == 2 ? 3 : 4))))
k_cells(const CellParams<R> p)
{
    constexpr int kTPB = kTX * kTY;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY, NB = N * PLANE;
    constexpr int NSH = N * N + P * N;  // staged per cell: x = 0 plane, then y = 0 row for x = 1..P
    __shared__ double sT[NB];
    __shared__ double sS[NSH * kTPB];
    __shared__ double sC[N * N * kTPB];  // carry: top-plane partial sums per lane, (y, x) major

    const int b = blockIdx.x;
    const int id = (b & 7) * p.tiles_per_xcd + (b >> 3);
    if (id >= p.ntiles) return;  // uniform over the workgroup
    const int seg = id % p.MZ, col = id / p.MZ;
    const int tx = col % p.MX, ty = col / p.MX;
    const int z0 = seg * p.seg_len, z1 = min(z0 + p.seg_len, p.nz);
    const int i0 = P * kTX * tx, j0 = P * kTY * ty;
    const int tpar = (tx & 1) | ((ty & 1) << 1) | ((seg & 1) << 2);
    const long long NXY = (long long)p.NX * p.NY, NT = NXY * p.NZ;

#pragma clang loop unroll(disable)
    for (int cz = z0; cz < z1; ++cz) {
        const int k0 = P * cz;
        // Everything derived from the lane index is recomputed inside the layer
        // loop: hoisting it would hold registers across the whole march.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        AS4<CellParams<R>> &q = *kernarg_params<CellParams<R>>();
        const Law<R> *lawp = q.law;
        const Law<double> *nlawp = q.nlaw;
        const int lx = tid % kTX, ly = tid / kTX;
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool active = cx < q.nx && cy < q.ny;
        // 1. stage the node planes of the layer
        for (int idx = tid; idx < NB; idx += kTPB) {
            const int li = idx % BX, lj = (idx / BX) % BY, lk = idx / PLANE;
            const int gi = i0 + li, gj = j0 + lj;
            double val = 0.0;
            if (gi < q.NX && gj < q.NY)
                val = q.Tin[(long long)gi + (long long)q.NX * gj + NXY * (k0 + lk)];
            sT[idx] = val;
        }
        __syncthreads();
        // 2. cell operator (every lane gathers, so that no value of a previous
        // layer stays live across the loop)
        R u[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
            const double tv = sT[(az * BY + P * ly + ay) * BX + P * lx + ax];
            if constexpr (std::is_same<R, double>::value) u[a] = tv;
            else u[a] = R(tv - q.Tref);
        }
        R fe[NN];
        if (active) {
            cell_operator<P, R>(q, lawp, u, cx, cy, cz, fe);
#pragma unroll
            for (int az = 0; az < N; ++az) {
#pragma unroll
                for (int ay = 0; ay < N; ++ay) sS[(az * N + ay) * kTPB + tid] = double(fe[(az * N + ay) * N]);
#pragma unroll
                for (int ax = 1; ax <= P; ++ax)
                    sS[(N * N + az * P + ax - 1) * kTPB + tid] = double(fe[az * N * N + ax]);
            }
        }
        __syncthreads();
        // 3. owned nodes: sum, carry, completion
        if (active) {
            const bool hasR = lx < kTX - 1 && cx + 1 < q.nx;
            const bool hasU = ly < kTY - 1 && cy + 1 < q.ny;
            const bool first = cz == z0, last = cz == z1 - 1;
#pragma unroll
            for (int az = 0; az < N; ++az) {
#pragma unroll
                for (int ay = 0; ay < N; ++ay) {
#pragma unroll
                    for (int ax = 0; ax < N; ++ax) {
                        if ((ax == 0 && lx != 0) || (ay == 0 && ly != 0)) continue;
                        double f = 0.0;
                        if (az == 0 && !first) f = sC[(ay * N + ax) * kTPB + tid];
                        f += double(fe[(az * N + ay) * N + ax]);
                        if (ax == P && hasR) f += sS[(az * N + ay) * kTPB + tid + 1];
                        if (ay == P && hasU)
                            f += ax == 0 ? sS[(az * N) * kTPB + tid + kTX]
                                         : sS[(N * N + az * P + ax - 1) * kTPB + tid + kTX];
                        if (ax == P && ay == P && hasR && hasU) f += sS[(az * N) * kTPB + tid + kTX + 1];
                        if (az == P && !last) {  // top plane: completed by the next layer
                            sC[(ay * N + ax) * kTPB + tid] = f;
                            continue;
                        }
                        const int gi = P * cx + ax, gj = P * cy + ay, gk = k0 + az;
                        const long long g = (long long)gi + (long long)q.NX * gj + NXY * gk;
                        const bool face = (az == 0 && first && gk > 0) || (az == P && last && gk < q.NZ - 1) ||
                                          is_face(gi, P * kTX, q.NX) || is_face(gj, P * kTY, q.NY);
                        if (face) {
                            q.slots[tpar * NT + g] = f;
                            continue;
                        }
                        const double T = sT[(az * BY + P * ly + ay) * BX + P * lx + ax];
                        const double C = node_capacity(const_law(nlawp), T, gi, gj, gk, P, q.NX, q.NY,
                                                       q.NZ, q.hx, q.hy, q.hz);
                        if (MODE == 0) {
                            q.Tout[g] = on_dirichlet(q.dmask, gi, gj, gk, q.NX, q.NY, q.NZ) ? q.T_D
                                                                                            : T + q.dt * f / C;
                        } else {
                            q.fout[g] = f;
                            q.Cout[g] = C;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Completion of the nodes on interior tile faces: fixed-order sum of the
// parity-slot partials of the (up to 8) tiles that contain the node.
template <int MODE>
__global__ void __launch_bounds__(256) k_halo(const HaloParams h)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long r = t;
    int gi, gj, gk, grp;
    if (r < h.GX) {  // x-faces: i = m*SX, m = 1..MX-1
        grp = 0;
        gj = int(r % h.NY);
        r /= h.NY;
        gk = int(r % h.NZ);
        gi = int(r / h.NZ + 1) * h.SX;
    } else if ((r -= h.GX) < h.GY) {  // y-faces without x-face nodes
        grp = 1;
        gi = int(r % h.NX);
        r /= h.NX;
        gk = int(r % h.NZ);
        gj = int(r / h.NZ + 1) * h.SY;
    } else if ((r -= h.GY) < h.GZ) {  // z-faces without x- or y-face nodes
        grp = 2;
        gi = int(r % h.NX);
        r /= h.NX;
        gj = int(r % h.NY);
        gk = int(r / h.NY + 1) * h.SZ;
    } else {
        return;
    }
    const bool fx = is_face(gi, h.SX, h.NX), fy = is_face(gj, h.SY, h.NY);
    if (grp == 0 && !fx) return;
    if (grp >= 1 && fx) return;
    if (grp == 1 && !fy) return;
    if (grp == 2 && (fy || !is_face(gk, h.SZ, h.NZ))) return;
    const bool fz = is_face(gk, h.SZ, h.NZ);
    // tiles containing the node along each direction
    int xs[2], ys[2], zs[2];
    int nxs, nys, nzs;
    if (fx) { xs[0] = gi / h.SX - 1; xs[1] = gi / h.SX; nxs = 2; } else { xs[0] = min(gi / h.SX, h.MX - 1); nxs = 1; }
    if (fy) { ys[0] = gj / h.SY - 1; ys[1] = gj / h.SY; nys = 2; } else { ys[0] = min(gj / h.SY, h.MY - 1); nys = 1; }
    if (fz) { zs[0] = gk / h.SZ - 1; zs[1] = gk / h.SZ; nzs = 2; } else { zs[0] = min(gk / h.SZ, h.MZ - 1); nzs = 1; }
    const long long NXY = (long long)h.NX * h.NY, NT = NXY * h.NZ;
    const long long g = (long long)gi + (long long)h.NX * gj + NXY * gk;
    double f = 0.0;
    for (int a = 0; a < nzs; ++a)
        for (int bb = 0; bb < nys; ++bb)
            for (int e = 0; e < nxs; ++e) {
                const int par = (xs[e] & 1) | ((ys[bb] & 1) << 1) | ((zs[a] & 1) << 2);
                f += h.slots[par * NT + g];
            }
    const double T = h.Tin[g];
    const double C = node_capacity(const_law(h.nlaw), T, gi, gj, gk, h.P, h.NX, h.NY, h.NZ, h.hx,
                                   h.hy, h.hz);
    if (MODE == 0) {
        h.Tout[g] = on_dirichlet(h.dmask, gi, gj, gk, h.NX, h.NY, h.NZ) ? h.T_D : T + h.dt * f / C;
    } else {
        h.fout[g] = f;
        h.Cout[g] = C;
    }
}

}  // namespace

namespace {
template <int TY>
void launch_ty(int degree, int precision, int mode, const CellParams<double> &pd,
               const CellParams<float> &pf, hipStream_t s)
{
    const int tpx = precision == PBF_PREC_FP32 ? pf.tiles_per_xcd : pd.tiles_per_xcd;
    const dim3 grid(8 * tpx), block(kTX * TY);
#define PBF_LAUNCH(P_, R_, M_, prm) hipLaunchKernelGGL((k_cells<P_, R_, M_, TY>), grid, block, 0, s, prm)
    if (precision == PBF_PREC_FP64) {
        if (degree == 1) { if (mode == 0) PBF_LAUNCH(1, double, 0, pd); else PBF_LAUNCH(1, double, 1, pd); }
        else { if (mode == 0) PBF_LAUNCH(2, double, 0, pd); else PBF_LAUNCH(2, double, 1, pd); }
    } else {
        if (degree == 1) { if (mode == 0) PBF_LAUNCH(1, float, 0, pf); else PBF_LAUNCH(1, float, 1, pf); }
        else { if (mode == 0) PBF_LAUNCH(2, float, 0, pf); else PBF_LAUNCH(2, float, 1, pf); }
    }
#undef PBF_LAUNCH
}
}  // namespace

// 16 x 16 cells per column workgroup: measured fastest of 16x4, 16x8 and 16x16
// on cfg2-size boxes (fewer column-face nodes, same per-lane work)
int column_height() { return 16; }

int resident_columns_per_cu(int ty) { return ty == 4 ? 8 : (ty == 8 ? 4 : 2); }

hipError_t launch_cells(int degree, int precision, int mode, int ty, const CellParams<double> &pd,
                        const CellParams<float> &pf, hipStream_t s)
{
    if (ty == 4) launch_ty<4>(degree, precision, mode, pd, pf, s);
    else if (ty == 8) launch_ty<8>(degree, precision, mode, pd, pf, s);
    else launch_ty<16>(degree, precision, mode, pd, pf, s);
    return hipGetLastError();
}

hipError_t launch_halo(int mode, const HaloParams &hp, hipStream_t s)
{
    const long long n = hp.GX + hp.GY + hp.GZ;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (mode == 0) hipLaunchKernelGGL(k_halo<0>, grid, block, 0, s, hp);
    else hipLaunchKernelGGL(k_halo<1>, grid, block, 0, s, hp);
    return hipGetLastError();
}

}  // namespace pbf
