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

#include "cellkit.h"

namespace pbf {
namespace {

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
                        if (p.hist_write) p.hist[hi] = double(g);
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
            stage_shared<P, kTPB>(sS, fe, tid);
        }
        __syncthreads();
        // 3. owned nodes: sum, carry, completion
        if (active) {
            owner_nodes<P, kTY>(fe, sS, sC, tid, lx, ly, cx, cy, q.nx, q.ny, k0, cz == z0, cz == z1 - 1,
                                q.NX, q.NY, q.NZ, q.slots + tpar * NT, NXY,
                                [&](long long g, int gi, int gj, int gk, int ax, int ay, int az, double f) {
                const double T = sT[(az * BY + P * ly + ay) * BX + P * lx + ax];
                const double C = node_capacity(const_law(nlawp), T, gi, gj, gk, P, q.NX, q.NY, q.NZ,
                                               q.hx, q.hy, q.hz);
                if (MODE == 0) {
                    q.Tout[g] = on_dirichlet(q.dmask, gi, gj, gk, q.NX, q.NY, q.NZ) ? q.T_D
                                                                                    : T + q.dt * f / C;
                } else {
                    q.fout[g] = f;
                    q.Cout[g] = C;
                }
            });
        }
        __syncthreads();
    }
}

// Completion of the nodes on column faces and segment ends: fixed-order sum of
// the parity-slot partials of the (up to 8) columns/segments that contain them.
template <int MODE>
__global__ void __launch_bounds__(256) k_halo(const HaloParams h)
{
    FaceNode fn;
    if (!face_node((long long)blockIdx.x * blockDim.x + threadIdx.x, h, fn)) return;
    const long long NT = (long long)h.NX * h.NY * h.NZ;
    const long long g = (long long)fn.gi + (long long)h.NX * fn.gj + (long long)h.NX * h.NY * fn.gk;
    double f = 0.0;
    for (int a = 0; a < fn.n; ++a) f += h.slots[fn.par[a] * NT + g];
    const double T = h.Tin[g];
    const double C = node_capacity(const_law(h.nlaw), T, fn.gi, fn.gj, fn.gk, h.P, h.NX, h.NY, h.NZ,
                                   h.hx, h.hy, h.hz);
    if (MODE == 0) {
        h.Tout[g] = on_dirichlet(h.dmask, fn.gi, fn.gj, fn.gk, h.NX, h.NY, h.NZ) ? h.T_D
                                                                                : T + h.dt * f / C;
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
