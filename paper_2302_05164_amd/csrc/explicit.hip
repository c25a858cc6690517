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
#include <hip/hip_ext.h>

#include "cellkit.h"

namespace pbf {
namespace {

// Exponent beyond which the volume source is skipped in a cell (e^-56 < 2^-80).
constexpr double kSourceCut = 56.0;

// Flux and source at the Gauss points of one cell, accumulated into the
// collocation-space integrand w.  FAST: at most one hinge of the law active, no
// source and no history update in the wave (uniform branch-free straight-line
// code); FHIST: the FAST cell reads its (unchanged) consolidated fraction.
template <int P, typename R, bool FAST, bool FHIST = false, typename PP, typename L>
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
    // General cells: the hinge sums of all points first, one hinge at a time
    // (each coefficient is read once per cell; every point still adds its
    // hinges in increasing order), and the Gaussian source once per (x, y)
    // column of points (its exponent does not depend on z).
    R kq[FAST ? 1 : NN];
    double sq[FAST ? 1 : N * N];
    if constexpr (!FAST) {
#pragma unroll
        for (int q = 0; q < NN; ++q) kq[q] = k0;
        for (int i = 0; i < nhinge; ++i) {
            const R bi = law.b[i], dki = law.dk[i];
#pragma unroll
            for (int q = 0; q < NN; ++q) kq[q] = ffma(dki, fmax0(v[q] - bi, R(0)), kq[q]);
        }
        if (src_cell) {
            sfor<0, N * N>([&](auto ic) {
                constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
                constexpr double xiq = TB::gp(i), etq = TB::gp(j);  // folded at compile time
                const double dxb = (cx + xiq) * p.hx - p.xb;
                const double dyb = (cy + etq) * p.hy - p.yb;
                sq[decltype(ic)::value] = p.src_amp * exp(-(dxb * dxb + dyb * dyb) * p.two_over_R2);
            });
        }
    }
    // general cells: the history of a z-plane of points, loaded together before
    // the plane (the updates would otherwise order each point's load behind the
    // previous point's store)
    R rpl[FAST ? 1 : N * N];
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
        if constexpr (!FAST && qx == 0 && qy == 0) {
            if (has_hist) {
#pragma unroll
                for (int j = 0; j < N * N; ++j) rpl[j] = R(p.hist[(long long)(qz * N * N + j) * p.n_hist_cells + hc]);
            }
        }
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
            if constexpr (FHIST) {
                const R r = R(p.hist[(long long)q * p.n_hist_cells + hc]);
                k = k * (r + law.phi * (R(1) - r));
            }
        } else {
            const R kpl = kq[q];
            k = kpl;
            if (has_hist) {
                const long long hi = (long long)q * p.n_hist_cells + hc;
                R r = rpl[qy * N + qx];
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
                constexpr double zeq = TB::gp(qz);
                const double zq = (cz + zeq) * p.hz;
                const double depth = p.Lz - zq;
                if (depth >= 0.0 && depth <= p.h_powder) w[q] = ffma(R(wq) * detJ, R(sq[qy * N + qx]), w[q]);
            }
        }
    });
}

// Unit-conductivity diffusion at the Gauss points (the constant-coefficient
// Laplace operator y = K x): flux W J^{-1} J^{-T} grad u, collocation transpose.
template <int P, typename R, typename PP>
__device__ __forceinline__ void flux_points_laplace(PP &p, const R *v, R *w)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    const R cx = p.detJ * p.ih2x, cy = p.detJ * p.ih2y, cz = p.detJ * p.ih2z;
    sfor<0, NN>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
        auto gxf = [&](auto rc) { return v[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
        auto gyf = [&](auto rc) { return v[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
        auto gzf = [&](auto rc) { return v[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
        constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
        const R Fx = R(wq) * cx * rowdot<TagD<P>, qx, 0, N, false>(gxf, R(0));
        const R Fy = R(wq) * cy * rowdot<TagD<P>, qy, 0, N, false>(gyf, R(0));
        const R Fz = R(wq) * cz * rowdot<TagD<P>, qz, 0, N, false>(gzf, R(0));
        sfor<0, N>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
            if constexpr (dx != 0.0) w[tidx<N, 0>(r, qy, qz)] = ffma(R(dx), Fx, w[tidx<N, 0>(r, qy, qz)]);
            if constexpr (dy != 0.0) w[tidx<N, 1>(r, qx, qz)] = ffma(R(dy), Fy, w[tidx<N, 1>(r, qx, qz)]);
            if constexpr (dz != 0.0) w[tidx<N, 2>(r, qx, qy)] = ffma(R(dz), Fz, w[tidx<N, 2>(r, qx, qy)]);
        });
    });
}

// ---------------------------------------------------------------------------
// one cell: nodal values u -> element vector fe (diffusion, source, surface
// flux).  Values are relative to Tref (zero in double precision).  MODE 2:
// the unit-conductivity Laplace operator alone.
// ---------------------------------------------------------------------------
template <int P, typename R, int MODE, typename PP>
__device__ __forceinline__ void cell_operator(PP &p, const Law<R> *lawp, const R *u, int cx, int cy,
                                              int cz, R *fe)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    R t1[NN], t2[NN], v[NN];
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, v);  // values at the Gauss points
    if constexpr (MODE == 2) {
        R w[NN];
#pragma unroll
        for (int q = 0; q < NN; ++q) w[q] = R(0);
        flux_points_laplace<P, R>(p, v, w);
        sweep<TagSt<P>, N, 0>(w, t1);
        sweep<TagSt<P>, N, 1>(t1, t2);
        sweep<TagSt<P>, N, 2>(t2, fe);
        return;
    }

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
    bool src_cell = p.laser_on && p.laser_kind == 1 && cz >= p.src_cz0;
    if (src_cell) {
        // Gauss points at least as far from the beam axis as the cell's box.
        // Where the Gaussian's exponent is below -kSourceCut the source is
        // below e^-56 (< 2^-80) of its peak at every point of the cell: the
        // temperature increment it would add in a step is that fraction of the
        // peak increment, far below the rounding unit of any temperature
        const double ex = fmax(0.0, fmax(cx * p.hx - p.xb, p.xb - (cx + 1) * p.hx));
        const double ey = fmax(0.0, fmax(cy * p.hy - p.yb, p.yb - (cy + 1) * p.hy));
        src_cell = (ex * ex + ey * ey) * p.two_over_R2 < kSourceCut;
    }

    R w[NN];  // collocation-space integrand of f
#pragma unroll
    for (int q = 0; q < NN; ++q) w[q] = R(0);
    // Most cells of a scan are cold and away from the beam: for them the points
    // run as one straight-line block (one hinge at most, no source, no history
    // update), which lets the scheduler interleave independent points.  All
    // paths evaluate the same arithmetic.
    // (a wave with a source cell takes the general path as a whole: running
    // both paths under masks would cost their sum)
    if (nhinge <= 1 && !__any(src_cell) && !(has_hist && melt)) {
        if (has_hist)
            flux_points<P, R, true, true>(p, law, v, w, nhinge, false, true, hc, false, cx, cy, cz);
        else
            flux_points<P, R, true>(p, law, v, w, nhinge, false, false, 0, false, cx, cy, cz);
    } else
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

// Owner-computes completion of the nodes of one cell layer (explicit step or
// assembly).  The lane of cell (lx, ly) owns the nodes of its cell with local
// x and y in 1..P (plus 0 on the column's low faces).  The sum order of every
// node is fixed: carry (cells below), own, right, upper, diagonal neighbour.
// Top-plane sums are carried in sC to the next layer; nodes on column faces and
// segment ends go to the parity slot array; the others are completed here.
// Everything is straight-line per lane: the law constants are read once, the
// capacity hinges are truncated once per layer to those that some node of the
// wave exceeds, and every node ends in one store through a selected address.
template <int P, int kTY, int MODE, typename Q, typename R>
__device__ __forceinline__ void owner_update(Q &q, const R *fe, const double *sS, double *sC,
                                             const double *sTl, int r0, int tid, int lx, int ly,
                                             int cx, int cy, int k0, int seg, bool first, bool last,
                                             double *slots, long long NXY)
{
    constexpr int N = P + 1, kTPB = kTX * kTY;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY;
    const bool hasR = lx < kTX - 1 && cx + 1 < q.nx;
    const bool hasU = ly < kTY - 1 && cy + 1 < q.ny;
    const double *sTz[N];  // node plane az of the layer (rotating slots)
#pragma unroll
    for (int az = 0; az < N; ++az) sTz[az] = sTl + (r0 + az < N ? r0 + az : r0 + az - N) * PLANE;
    ConstLaw<double> &L = const_law(q.nlaw);
    // capacity hinges that some node of the wave exceeds (hinges above every
    // node add exactly zero)
    int nh = 0;
    if constexpr (MODE != 2) {
        double tmax = sTz[0][0];
#pragma unroll
        for (int a = 1; a < N * N * N; ++a) tmax = fmax(tmax, sTz[a / (N * N)][((a / N) % N) * BX + a % N]);
        while (nh < L.n_hinge && __any(tmax > L.b[nh])) ++nh;
    }
    const double c0 = L.c0, Ts = L.Ts, Tl = L.Tl, lat = L.lat, rho = L.rho;
    const int NX = q.NX, NY = q.NY, NZ = q.NZ;
    const unsigned dmask = q.dmask;
    const double hx = q.hx, hy = q.hy, hz = q.hz, dt = q.dt, T_D = q.T_D;
    const FaceMap fm = face_map_of(q);
    // nodes with local y = 0 belong to the lanes of the column's first row only
    // (all in the first wavefront): the other wavefronts skip them as a whole
    const bool has_row0 = __builtin_amdgcn_readfirstlane(tid) < kTX;
#pragma unroll
    for (int az = 0; az < N; ++az) {
        // capacities of the plane's nodes, one hinge at a time (each law
        // coefficient read once per plane; every node adds its hinges in
        // increasing order)
        double cpl[N * N];
        if (MODE != 2 && (az < P || last)) {
#pragma unroll
            for (int j = 0; j < N * N; ++j) {
                const double T = sTz[az][(j / N) * BX + j % N];
                cpl[j] = c0 + ((T >= Ts && T <= Tl) ? lat : 0.0);
            }
            for (int h = 0; h < nh; ++h) {
                const double bh = L.b[h], dch = L.dc[h];
#pragma unroll
                for (int j = 0; j < N * N; ++j)
                    cpl[j] = __builtin_fma(dch, fmax0(sTz[az][(j / N) * BX + j % N] - bh, 0.0), cpl[j]);
            }
        }
#pragma unroll
        for (int ay = 0; ay < N; ++ay) {
            if (ay == 0 && !has_row0) continue;  // uniform
#pragma unroll
            for (int ax = 0; ax < N; ++ax) {
                const int n = (az * N + ay) * N + ax;
                double f = 0.0;
                if (az == 0 && !first) f = sC[(ay * N + ax) * kTPB + tid];
                f += double(fe[n]);
                if (ax == P) {
                    const double r = sS[(az * N + ay) * kTPB + tid + 1];
                    f += hasR ? r : 0.0;
                }
                if (ay == P) {
                    const double u = ax == 0 ? sS[(az * N) * kTPB + tid + kTX]
                                             : sS[(N * N + az * P + ax - 1) * kTPB + tid + kTX];
                    f += hasU ? u : 0.0;
                }
                if (ax == P && ay == P) {
                    const double d = sS[(az * N) * kTPB + tid + kTX + 1];
                    f += (hasR && hasU) ? d : 0.0;
                }
                if (az == P && !last) {  // uniform: completed by the next layer
                    sC[(ay * N + ax) * kTPB + tid] = f;
                    continue;
                }
                const bool own = (ax != 0 || lx == 0) && (ay != 0 || ly == 0);
                const int gi = P * cx + ax, gj = P * cy + ay, gk = k0 + az;
                const long long g = (long long)gi + (long long)NX * gj + NXY * gk;
                const bool face = (az == 0 && first && gk > 0) || (az == P && last && gk < NZ - 1) ||
                                  is_face(gi, P * kTX, NX) || is_face(gj, P * kTY, NY);
                const double T = sTz[az][ay * BX + ax];
                const double c = cpl[ay * N + ax];
                const double m = lumped_mass_1d(gi, NX, P, hx) * lumped_mass_1d(gj, NY, P, hy) *
                                 lumped_mass_1d(gk, NZ, P, hz);
                const double C = rho * c * m;
                const long long t = face_slot(gi, gj, gk, az == 0 ? seg - 1 : seg, P * kTX, P * kTY, NX, NY, NZ, fm);
                if (MODE == 0) {
                    // face nodes: the lowest containing column (the first term of the face
                    // kernel's fixed-order sum) stores its complete update, the others only
                    // their increment, so the face kernel needs neither T_n nor C~
                    const bool dir = on_dirichlet(dmask, gi, gj, gk, NX, NY, NZ);
                    const double inc = dt * f / C;
                    const bool later = (ax == 0 && is_face(gi, P * kTX, NX)) ||
                                       (ay == 0 && is_face(gj, P * kTY, NY)) || (az == 0 && first && gk > 0);
                    const double val = dir ? ((face && later) ? 0.0 : T_D) : ((face && later) ? inc : T + inc);
                    double *dst = face ? slots + t : q.Tout + g;
                    if (own) *dst = val;
                } else {
                    double *dst = face ? slots + t : q.fout + g;
                    if (own) *dst = f;
                    if (MODE == 1 && own && !face) q.Cout[g] = C;
                }
            }
        }
    }
}

// MODE 0: explicit step (fused update into Tout); MODE 1: assemble f and C~;
// MODE 2: the unit-conductivity Laplace operator y = K x into fout.
//
// Node ownership inside a column: the lane of cell (lx, ly) owns the nodes of
// its cell with local x and y indices in 1..P (plus index 0 on the column's
// low faces).  Own contributions come straight from registers; the shared
// contributions of the right, upper and diagonal neighbour cells come from a
// small LDS staging area (each cell stages its x = 0 plane and its y = 0 row);
// the top node plane is carried per lane to the next layer.  The sum order of
// every node is fixed: carry, own, right, upper, diagonal.
//
// Node planes live in N rotating LDS slots (global plane k in slot k mod N):
// the top plane of a layer stays resident as the bottom plane of the next, and
// the P new planes of the next layer are loaded into registers before the
// node completion of the current one (which hides their latency) and stored
// into the slots of the planes that layer no longer needs.
template <int P, typename R, int MODE, int kTY>
__global__ void __launch_bounds__(kTX * kTY) __attribute__((amdgpu_waves_per_eu(P == 2 && sizeof(R) == 8 ? 2 : (P == 2 ? 3 : 4))))
k_cells(const CellParams<R> p)
{
    constexpr int kTPB = kTX * kTY;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY, NB = N * PLANE;
    constexpr int NSH = N * N + P * N;  // staged per cell: x = 0 plane, then y = 0 row for x = 1..P
    constexpr int NPF = (P * PLANE + kTPB - 1) / kTPB;  // prefetched values per lane
    __shared__ double sT[NB];
    __shared__ double sS[NSH * kTPB + kTX + 1];  // padded: neighbour reads of edge lanes stay inside
    __shared__ double sC[N * N * kTPB];  // carry: top-plane partial sums per lane, (y, x) major

    // Each XCD owns a contiguous range of tiles (whole columns when the range
    // is a multiple of the segment count).  Within it the top segments, which
    // hold the powder layer, the beam and the hottest cells, are dispatched
    // first: the first workgroup on a CU is the older one and wins the issue
    // arbitration against a later one, which shortens the critical path.
    const int b = blockIdx.x;
    const int xcd = b & 7, j = b >> 3;
    int id = xcd * p.tiles_per_xcd + j;
    if (p.tiles_per_xcd % p.MZ == 0) {
        const int cpx = p.tiles_per_xcd / p.MZ;
        id = (xcd * cpx + j % cpx) * p.MZ + (p.MZ - 1 - j / cpx);
    }
    if (id >= p.ntiles) return;  // uniform over the workgroup
    const int seg = id % p.MZ, col = id / p.MZ;
    const int tx = col % p.MX, ty = col / p.MX;
    const int z0 = p.zb[seg], z1 = p.zb[seg + 1];
    const int i0 = P * kTX * tx, j0 = P * kTY * ty;
    const int tpar = (tx & 1) | ((ty & 1) << 1) | ((seg & 1) << 2);
    const long long NXY = (long long)p.NX * p.NY;

    // the N node planes of the first layer: every load of the lane is issued
    // before the first store, so the latencies overlap
    {
        constexpr int NL = (NB + kTPB - 1) / kTPB;
        double val[NL];
#pragma unroll
        for (int e = 0; e < NL; ++e) {
            const unsigned idx = threadIdx.x + unsigned(e * kTPB);
            const unsigned lp = idx / PLANE, rem = idx - lp * PLANE;
            const unsigned li = rem % BX, lj = rem / BX;
            const int gi = i0 + int(li), gj = j0 + int(lj), gk = P * z0 + int(lp);
            val[e] = 0.0;
            if (idx < unsigned(NB) && gi < p.NX && gj < p.NY)
                val[e] = p.Tin[(long long)gi + (long long)p.NX * gj + NXY * gk];
        }
#pragma unroll
        for (int e = 0; e < NL; ++e) {
            const unsigned idx = threadIdx.x + unsigned(e * kTPB);
            const unsigned lp = idx / PLANE, rem = idx - lp * PLANE;
            if (idx < unsigned(NB)) sT[((P * z0 + int(lp)) % N) * PLANE + rem] = val[e];
        }
    }
    __syncthreads();

#pragma clang loop unroll(disable)
    for (int cz = z0; cz < z1; ++cz) {
        const int k0 = P * cz, r0 = k0 % N;
        // Everything derived from the lane index is recomputed inside the layer
        // loop: hoisting it would hold registers across the whole march.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        AS4<CellParams<R>> &q = *kernarg_params<CellParams<R>>();
        const Law<R> *lawp = q.law;
        const int lx = tid % kTX, ly = tid / kTX;
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool active = cx < q.nx && cy < q.ny;
        const double *sTl = sT + P * (ly * BX + lx);  // node (0,0,.) of the lane's cell
        // 1. cell operator (every lane gathers, so that no value of a previous
        // layer stays live across the loop)
        R u[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
            const int sl = r0 + az < N ? r0 + az : r0 + az - N;
            const double tv = sTl[sl * PLANE + ay * BX + ax];
            if constexpr (std::is_same<R, double>::value) u[a] = tv;
            else u[a] = R(tv - q.Tref);
        }
        R fe[NN];
        if (active) {
            cell_operator<P, R, MODE>(q, lawp, u, cx, cy, cz, fe);
            if (MODE != 2 && q.re.on && cz == q.nz - 1) {  // top face: radiation and evaporation
                const int st = r0 + P < N ? r0 + P : r0 + P - N;
                const double *top = sTl + st * PLANE;
                surface_loss_face<P>(q.re, q.hx, q.hy, [&](int ax, int ay) { return top[ay * BX + ax]; }, fe);
            }
            stage_shared<P, kTPB>(sS, fe, tid);
        }
        __syncthreads();
        // 2. loads of the next layer's new planes (global planes k0+N .. k0+N+P-1)
        const bool more = cz + 1 < z1;
        double pf[NPF];
        if (more) {
#pragma unroll
            for (int e = 0; e < NPF; ++e) {
                const unsigned idx = unsigned(tid) + unsigned(e * kTPB);
                pf[e] = 0.0;
                if (idx < unsigned(P * PLANE)) {
                    const unsigned lp = idx / PLANE, rem = idx - lp * PLANE;
                    const unsigned li = rem % BX, lj = rem / BX;
                    const int gi = i0 + int(li), gj = j0 + int(lj);
                    if (gi < q.NX && gj < q.NY)
                        pf[e] = q.Tin[(long long)gi + (long long)q.NX * gj + NXY * (k0 + N + int(lp))];
                }
            }
        }
        // 3. owned nodes: sum, carry, completion
        if (active) {
            owner_update<P, kTY, MODE>(q, fe, sS, sC, sTl, r0, tid, lx, ly, cx, cy, k0, seg, cz == z0,
                                       cz == z1 - 1, q.slots + tpar * q.fm.GT, NXY);
        }
        __syncthreads();
        // 4. the new planes replace planes k0 .. k0+P-1 (slots r0 .. r0+P-1 mod N)
        if (more) {
#pragma unroll
            for (int e = 0; e < NPF; ++e) {
                const unsigned idx = unsigned(tid) + unsigned(e * kTPB);
                if (idx < unsigned(P * PLANE)) {
                    const unsigned lp = idx / PLANE, rem = idx - lp * PLANE;
                    const int sl = r0 + int(lp) < N ? r0 + int(lp) : r0 + int(lp) - N;
                    sT[sl * PLANE + rem] = pf[e];
                }
            }
            __syncthreads();
        }
    }
}

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

template <int TY>
void launch_ty(int degree, int precision, int mode, const CellParams<double> &pd,
               const CellParams<float> &pf, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const int tpx = precision == PBF_PREC_FP32 ? pf.tiles_per_xcd : pd.tiles_per_xcd;
    const dim3 grid(8 * tpx), block(kTX * TY);
#define PBF_LAUNCH(P_, R_, M_, prm) launch_maybe_timed(k_cells<P_, R_, M_, TY>, grid, block, s, e0, e1, prm)
    if (precision == PBF_PREC_FP64) {
        if (degree == 1) {
            if (mode == 0) PBF_LAUNCH(1, double, 0, pd);
            else if (mode == 1) PBF_LAUNCH(1, double, 1, pd);
            else PBF_LAUNCH(1, double, 2, pd);
        } else {
            if (mode == 0) PBF_LAUNCH(2, double, 0, pd);
            else if (mode == 1) PBF_LAUNCH(2, double, 1, pd);
            else PBF_LAUNCH(2, double, 2, pd);
        }
    } else {
        if (degree == 1) { if (mode == 0) PBF_LAUNCH(1, float, 0, pf); else PBF_LAUNCH(1, float, 1, pf); }
        else { if (mode == 0) PBF_LAUNCH(2, float, 0, pf); else PBF_LAUNCH(2, float, 1, pf); }
    }
#undef PBF_LAUNCH
}
}  // namespace

// 16 x 16 cells per column workgroup: measured fastest of 16x4, 16x8 and 16x16
// on 128x128x64 and 48x48x24 Q2 boxes (fewer column-face nodes, same per-lane work)
int column_height() { return 16; }

int resident_columns_per_cu(int ty) { return ty == 4 ? 8 : (ty == 8 ? 4 : 2); }

hipError_t launch_cells(int degree, int precision, int mode, int ty, const CellParams<double> &pd,
                        const CellParams<float> &pf, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (ty == 4) launch_ty<4>(degree, precision, mode, pd, pf, s, e0, e1);
    else if (ty == 8) launch_ty<8>(degree, precision, mode, pd, pf, s, e0, e1);
    else launch_ty<16>(degree, precision, mode, pd, pf, s, e0, e1);
    return hipGetLastError();
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
