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
#pragma once
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
template <int P, typename R, bool FAST, bool FHIST = false, bool ISO = false, typename PP, typename L>
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
    const R ndih = ISO ? -(detJ * ih2x) : R(0);
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
        // flux -k W J^{-1} J^{-T} grad T, collocation transpose (ISO: equal
        // spacing in x, y and z, one common factor -W detJ / h^2 per point)
        R Fx, Fy, Fz;
        if constexpr (ISO) {
            const R kWi = k * (R(wq) * ndih);
            Fx = kWi * gx;
            Fy = kWi * gy;
            Fz = kWi * gz;
        } else {
            const R kW = k * (R(wq) * detJ);
            Fx = -kW * ih2x * gx;
            Fy = -kW * ih2y * gy;
            Fz = -kW * ih2z * gz;
        }
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
            if (p.iso)
                flux_points<P, R, true, false, true>(p, law, v, w, nhinge, false, false, 0, false, cx, cy, cz);
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

// Lane mapping of node-plane loads and their LDS stores.  Regular elements:
// element e of a lane is plane e / P^2, row tid / W + RPP * (e % P^2) (RPP =
// kTPB / W rows per pass; the P^2 passes of a plane cover its rows 0 .. P*kTY-1
// exactly) at column tid % W, so that plane and row offset are compile-time
// constants per element and the lane's own part is fixed.  Extra elements: the
// last row (row P*kTY, columns 0 .. W-1) and the last column (column W, rows
// 0 .. P*kTY) of every plane, dealt out over the lanes.  Offsets are 32-bit,
// relative to the planes' first node (i0, j0, k); the caller checks that a
// column's planes fit in 32 bits.
template <int P, int kTY, int NP>
struct PlaneRows {
    static constexpr int W = P * kTX, BX = W + 1, BY = P * kTY + 1, kTPB = kTX * kTY;
    static constexpr int RPP = kTPB / W, PPP = P * P;
    static constexpr int NREG = NP * PPP;
    static constexpr int NEXTRA = (NP * (W + BY) + kTPB - 1) / kTPB;
    static_assert(RPP * PPP == BY - 1, "the regular passes cover all rows but the last");
    // extra element x of lane tid: plane lp, row lj, column li (false: none)
    __device__ static __forceinline__ bool extra(int tid, int x, int &lp, int &lj, int &li)
    {
        const int idx = tid + kTPB * x;
        if (idx < NP * W) {
            lp = idx / W;
            lj = BY - 1;
            li = idx % W;
            return true;
        }
        const int k = idx - NP * W;
        lp = k / BY;
        lj = k - lp * BY;
        li = W;
        return k < NP * BY;
    }
};

// 1/x for the positive, normal capacities of the update: hardware reciprocal
// refined by two Newton steps (relative error near one unit in the last place).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// 1/m of the 1D row-sum lumped mass (h (1/6, 2/3, 1/6) per Q2 cell, h (1/2, 1/2)
// per Q1 cell) at a node: midpoint, interior vertex or boundary vertex
template <int P>
__device__ __forceinline__ double inv_mass_1d(bool midpoint, bool boundary, double ih)
{
    if constexpr (P == 2) return (midpoint ? 1.5 : (boundary ? 6.0 : 3.0)) * ih;
    else return (boundary ? 2.0 : 1.0) * ih;
}

// Completion of the nodes of one cell layer (explicit step or assembly), in
// two parts that share one barrier after the LDS staging of the cell vectors.
//
// Interior nodes (column-local x and y index in 1..P*kTX-1 and 1..P*kTY-1): the
// lane of cell (lx, ly) owns its cell's nodes with local x and y in 1..P.  Their
// sum order is fixed: carry (cells below), own, right, upper, diagonal
// neighbour.  None of them lies on a column face, so every one is completed
// here (straight-line code: no face test, 32-bit offsets from the layer's
// base, a reciprocal instead of a division) except on the end planes of a
// segment, which go to the slot array as a whole.
//
// Perimeter nodes (column-local x or y index 0 or P*kTX, P*kTY): spread over
// all lanes, one (position, z-plane) item each; contributions of the (one to
// four) containing cells of the column in a fixed order (cells by y, then x),
// read from the staged x = 0 planes and y = 0 rows and from the staged high
// faces of the last row and column (sE); top-plane sums are carried in sPC
// (two buffers alternating by layer, since the item of a node's bottom plane
// and that of its top plane may run on different lanes).  Column-face and
// segment-end nodes store their partial sums to the slot array; boundary nodes
// of the domain are completed here.
template <int P, int kTY, int MODE, typename Q, typename R>
__device__ __forceinline__ void complete_layer(Q &q, const R *fe, const double *sS, const double *sE,
                                               double *sC, double *sPC, const double *sT, int r0, int tid,
                                               int lx, int ly, int tx, int ty, int cz, int seg, bool first,
                                               bool last, bool active, double *slots)
{
    constexpr int N = P + 1, kTPB = kTX * kTY;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY;
    constexpr int NPER = 2 * BY + 2 * (BX - 2);  // perimeter positions of a node plane
    ConstLaw<double> &L = const_law(q.nlaw);
    const int NX = q.NX, NY = q.NY, NZ = q.NZ;
    const int i0 = P * kTX * tx, j0 = P * kTY * ty, k0 = P * cz;
    const unsigned dmask = q.dmask;
    const double dtr = q.dtr, ihx = q.ihx, ihy = q.ihy, ihz = q.ihz;  // dt / rho, 1/h (uniform)
    int slot_r[N];  // node plane az of the layer (rotating slots)
#pragma unroll
    for (int az = 0; az < N; ++az) slot_r[az] = (r0 + az < N ? r0 + az : r0 + az - N) * PLANE;

    // ---------------- interior nodes ----------------
    if (active) {
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool hasR = cx + 1 < q.nx, hasU = cy + 1 < q.ny;  // right/upper cell exists
        const bool xin = lx < kTX - 1, yin = ly < kTY - 1;     // the ax = P / ay = P nodes are interior
        const bool bx = cx == q.nx - 1, by = cy == q.ny - 1;   // ... and on the domain's high boundary
        const double *sTl = sT + P * (ly * BX + lx);
        // capacity hinges that some node of the wave exceeds
        int nh = 0;
        if constexpr (MODE != 2) {
            double tmax = sTl[slot_r[0] + BX + 1];
#pragma unroll
            for (int az = 0; az < N; ++az)
#pragma unroll
                for (int ay = 1; ay < N; ++ay)
#pragma unroll
                    for (int ax = 1; ax < N; ++ax) tmax = fmax(tmax, sTl[slot_r[az] + ay * BX + ax]);
            while (nh < L.n_hinge && __any(tmax > L.b[nh])) ++nh;
        }
        const double c0 = L.c0, Ts = L.Ts, Tl = L.Tl, lat = L.lat;
        // base of the layer's nodes (uniform) and the lane's 32-bit offset
        // dt / rho times the inverse lumped masses in x and y of the lane's nodes
        double sxy[P * P];
        if constexpr (MODE == 0) {
#pragma unroll
            for (int ay = 1; ay < N; ++ay)
#pragma unroll
                for (int ax = 1; ax < N; ++ax)
                    sxy[(ay - 1) * P + ax - 1] = dtr * inv_mass_1d<P>(P == 2 && ax == 1, ax == P && bx, ihx) *
                                                 inv_mass_1d<P>(P == 2 && ay == 1, ay == P && by, ihy);
        }
        double *const out = MODE == 0 ? q.Tout : q.fout;
        const long long base = (long long)i0 + (long long)NX * j0 + (long long)NX * NY * k0;
        const unsigned NXY = unsigned(NX) * unsigned(NY);
        const unsigned lane_off = unsigned(P * lx) + unsigned(NX) * unsigned(P * ly);
#pragma unroll
        for (int az = 0; az < N; ++az) {
            if (az == P && !last) {  // uniform: partial sums carried to the next layer
#pragma unroll
                for (int ay = 1; ay < N; ++ay)
#pragma unroll
                    for (int ax = 1; ax < N; ++ax) {
                        const int n = (az * N + ay) * N + ax;
                        double f = double(fe[n]);
                        if (ax == P) f += hasR ? sS[(az * N + ay) * kTPB + tid + 1] : 0.0;
                        if (ay == P) f += hasU ? sS[(N * N + az * P + ax - 1) * kTPB + tid + kTX] : 0.0;
                        if (ax == P && ay == P) f += (hasR && hasU) ? sS[(az * N) * kTPB + tid + kTX + 1] : 0.0;
                        sC[(ay * N + ax) * kTPB + tid] = f;
                    }
                continue;
            }
            const int gk = k0 + az;
            // uniform over the workgroup: segment ends are column faces
            const bool zface = (az == 0 && first && gk > 0) || (az == P && last && gk < NZ - 1);
            const bool zlater = az == 0 && first && gk > 0;
            const bool zdir = ((dmask & 16u) && gk == 0) || ((dmask & 32u) && gk == NZ - 1);
            const double iz = inv_mass_1d<P>(P == 2 && az == 1, gk == 0 || gk == NZ - 1, ihz);
            const int zf = az == 0 ? seg - 1 : seg;
            // capacities of the plane's interior nodes, one hinge at a time (each
            // law coefficient read once per plane; every node adds its hinges in
            // increasing order)
            double cpl[P * P];
            if constexpr (MODE != 2) {
#pragma unroll
                for (int j = 0; j < P * P; ++j) {
                    const double T = sTl[slot_r[az] + (j / P + 1) * BX + j % P + 1];
                    cpl[j] = c0 + ((T >= Ts && T <= Tl) ? lat : 0.0);
                }
                for (int h = 0; h < nh; ++h) {
                    const double bh = L.b[h], dch = L.dc[h];
#pragma unroll
                    for (int j = 0; j < P * P; ++j)
                        cpl[j] = __builtin_fma(dch, fmax0(sTl[slot_r[az] + (j / P + 1) * BX + j % P + 1] - bh, 0.0), cpl[j]);
                }
            }
#pragma unroll
            for (int ay = 1; ay < N; ++ay) {
                if (ay == P && !yin) continue;
#pragma unroll
                for (int ax = 1; ax < N; ++ax) {
                    if (ax == P && !xin) continue;
                    const int n = (az * N + ay) * N + ax;
                    double f = 0.0;
                    if (az == 0 && !first) f = sC[(ay * N + ax) * kTPB + tid];
                    f += double(fe[n]);
                    if (ax == P) f += hasR ? sS[(az * N + ay) * kTPB + tid + 1] : 0.0;
                    if (ay == P) f += hasU ? sS[(N * N + az * P + ax - 1) * kTPB + tid + kTX] : 0.0;
                    if (ax == P && ay == P) f += (hasR && hasU) ? sS[(az * N) * kTPB + tid + kTX + 1] : 0.0;
                    const unsigned off = lane_off + unsigned(ax) + unsigned(NX) * unsigned(ay) + NXY * unsigned(az);
                    const bool dir = zdir || ((dmask & 2u) && bx && ax == P) || ((dmask & 8u) && by && ay == P);
                    if constexpr (MODE == 2) {
                        if (zface)
                            slots[q.fm.GX + q.fm.GY + ((long long)zf * NY + j0 + P * ly + ay) * NX + i0 + P * lx + ax] = f;
                        else
                            out[base + off] = f;
                        continue;
                    }
                    const double T = sTl[slot_r[az] + ay * BX + ax];
                    const double c = cpl[(ay - 1) * P + ax - 1];
                    if constexpr (MODE == 0) {
                        const double inc = f * (sxy[(ay - 1) * P + ax - 1] * iz) * rcp_nr(c);
                        if (zface) {
                            const double val = dir ? (zlater ? 0.0 : q.T_D) : (zlater ? inc : T + inc);
                            slots[q.fm.GX + q.fm.GY + ((long long)zf * NY + j0 + P * ly + ay) * NX + i0 + P * lx + ax] = val;
                        } else {
                            out[base + off] = dir ? q.T_D : T + inc;
                        }
                    } else {  // MODE 1
                        if (zface) {
                            slots[q.fm.GX + q.fm.GY + ((long long)zf * NY + j0 + P * ly + ay) * NX + i0 + P * lx + ax] = f;
                        } else {
                            const int gi = i0 + P * lx + ax, gj = j0 + P * ly + ay;
                            const double m = lumped_mass_1d(gi, NX, P, q.hx) * lumped_mass_1d(gj, NY, P, q.hy) *
                                             lumped_mass_1d(gk, NZ, P, q.hz);
                            out[base + off] = f;
                            q.Cout[base + off] = L.rho * c * m;
                        }
                    }
                }
            }
        }
    }

    // ---------------- perimeter nodes ----------------
    // One side of the column per wave, each side with one corner: x = 0
    // (y index 0 .. P*kTY-1), x = P*kTX (y index 1 .. P*kTY), y = 0 (x index
    // 1 .. P*kTX), y = P*kTY (x index 0 .. P*kTX-1), so that each wave runs one
    // straight-line variant over as many positions as it has lanes (Q2, 16x16
    // cells: 32 positions x 2 planes, plus the top plane on half the lanes).
    // Along a side, a node at index a lies in the cell below it, (a-1)/P, unless
    // a = 0, and in the cell above it, a/P, when a is a multiple of P and that
    // cell belongs to the column; the two are added in that order (cells by y,
    // then x).
    const double *pc_prev = sPC + ((cz & 1) ^ 1) * NPER;
    double *pc_cur = sPC + (cz & 1) * NPER;
    const FaceMap fm = face_map_of(q);
    constexpr int NWAVE = kTPB / 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6, lane = tid & 63;
    sfor<0, 4>([&](auto sc) {
        constexpr int S = decltype(sc)::value;
        if (S % NWAVE != wave) return;  // uniform
        constexpr bool XS = S < 2;       // nodes along y at fixed x
        constexpr int NPOS = XS ? P * kTY : P * kTX;
        constexpr int POS0 = S == 0 ? 0 : (S == 1 ? P * kTY : (S == 2 ? 2 * P * kTY : 2 * P * kTY + P * kTX));
        // contribution of cell c along the side, at index a (0..P) along the side
        auto part = [&](int az, int c, int a) -> double {
            if constexpr (S == 0) return sS[(az * N + a) * kTPB + kTX * c];
            else if constexpr (S == 1)
                return a == 0 ? sS[(N * N + az * P + P - 1) * kTPB + kTX - 1 + kTX * c]
                              : sE[(az * P + a - 1) * kTY + c];
            else if constexpr (S == 2)
                return a == 0 ? sS[(az * N) * kTPB + c] : sS[(N * N + az * P + a - 1) * kTPB + c];
            else
                return a == 0 ? sS[(az * N + P) * kTPB + kTX * (kTY - 1) + c]
                              : sE[P * N * kTY + (az * P + a - 1) * kTX + c];
        };
        for (int it = lane; it < NPOS * N; it += 64) {
            const int az = it / NPOS, pp = it - az * NPOS;
            const int li = S == 0 ? 0 : (S == 1 ? P * kTX : (S == 2 ? pp + 1 : pp));
            const int lj = S == 0 ? pp : (S == 1 ? pp + 1 : (S == 2 ? 0 : P * kTY));
            const int gi = i0 + li, gj = j0 + lj, gk = k0 + az;
            if (gi >= NX || gj >= NY) continue;
            const int pos = POS0 + pp;
            const int al = XS ? lj : li;  // index along the side
            double f = (az == 0 && !first) ? pc_prev[pos] : 0.0;
            if (al >= 1) {  // the cell below exists whenever the node does
                const int c = (al - 1) / P;
                f += part(az, c, al - P * c);
            }
            if (al % P == 0) {
                const int c = al / P;
                const bool ok = XS ? (c < kTY && kTY * ty + c < q.ny) : (c < kTX && kTX * tx + c < q.nx);
                if (ok) f += part(az, c, 0);
            }
            if (az == P && !last) {
                pc_cur[pos] = f;
                continue;
            }
            const bool fx = is_face(gi, P * kTX, NX), fy = is_face(gj, P * kTY, NY);
            const bool fz = (az == 0 && first && gk > 0) || (az == P && last && gk < NZ - 1);
            const bool face = fx || fy || fz;
            const long long g = (long long)gi + (long long)NX * gj + (long long)NX * NY * gk;
            const long long t = face_slot(gi, gj, gk, az == 0 ? seg - 1 : seg, P * kTX, P * kTY, NX, NY, NZ, fm);
            if constexpr (MODE == 2) {
                if (face) slots[t] = f;
                else q.fout[g] = f;
                continue;
            }
            const double T = sT[slot_r[az] + lj * BX + li];
            const double C = node_capacity(L, T, gi, gj, gk, P, NX, NY, NZ, q.hx, q.hy, q.hz);
            if constexpr (MODE == 0) {
                const bool dir = on_dirichlet(dmask, gi, gj, gk, NX, NY, NZ);
                const double inc = (q.dt * f) * rcp_nr(C);
                const bool later = (li == 0 && fx) || (lj == 0 && fy) || (az == 0 && first && gk > 0);
                const double val = dir ? ((face && later) ? 0.0 : q.T_D) : ((face && later) ? inc : T + inc);
                if (face) slots[t] = val;
                else q.Tout[g] = val;
            } else {
                if (face) slots[t] = f;
                else {
                    q.fout[g] = f;
                    q.Cout[g] = C;
                }
            }
        }
    });
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
    __shared__ double sT[NB];
    __shared__ double sS[NSH * kTPB + kTX + 1];  // padded: neighbour reads of edge lanes stay inside
    __shared__ double sC[N * N * kTPB];  // carry: top-plane partial sums per lane, (y, x) major
    // high faces of the column's last cell column (x = P, y = 1..P) and last cell
    // row (y = P, x = 1..P), for the perimeter nodes
    __shared__ double sE[P * N * (kTX + kTY)];
    __shared__ double sPC[2 * (2 * (P * kTY + 1) + 2 * (P * kTX - 1))];  // perimeter carries

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
        using PR = PlaneRows<P, kTY, N>;
        const double *src = p.Tin + ((long long)i0 + (long long)p.NX * j0 + NXY * (P * z0));
        const int nxl = p.NX - i0, nyl = p.NY - j0;
        const int rl = threadIdx.x / PR::W, cl = threadIdx.x % PR::W;
        const unsigned goff = unsigned(rl) * unsigned(p.NX) + unsigned(cl);
        double val[PR::NREG], vx[PR::NEXTRA];
#pragma unroll
        for (int e = 0; e < PR::NREG; ++e) {
            const int lp = e / PR::PPP, dr = PR::RPP * (e % PR::PPP);
            val[e] = 0.0;
            if (cl < nxl && rl + dr < nyl)
                val[e] = src[goff + unsigned(lp) * unsigned(NXY) + unsigned(dr) * unsigned(p.NX)];
        }
#pragma unroll
        for (int x = 0; x < PR::NEXTRA; ++x) {
            int lp, lj, li;
            const bool ok = PR::extra(threadIdx.x, x, lp, lj, li);
            vx[x] = 0.0;
            if (ok && li < nxl && lj < nyl)
                vx[x] = src[unsigned(lp) * unsigned(NXY) + unsigned(lj) * unsigned(p.NX) + unsigned(li)];
        }
        const int loff = rl * BX + cl;
#pragma unroll
        for (int e = 0; e < PR::NREG; ++e) {
            const int lp = e / PR::PPP, dr = PR::RPP * (e % PR::PPP);
            sT[((P * z0 + lp) % N) * PLANE + loff + dr * BX] = val[e];
        }
#pragma unroll
        for (int x = 0; x < PR::NEXTRA; ++x) {
            int lp, lj, li;
            if (PR::extra(threadIdx.x, x, lp, lj, li)) sT[((P * z0 + lp) % N) * PLANE + lj * BX + li] = vx[x];
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
            // Wave priority: the cell operator is dense FP64 arithmetic and runs
            // at the default priority; the staging (1) and the node completion
            // (2) are short, latency-bound chains of LDS and memory accesses, so
            // they issue ahead of the other workgroup's cell operator on the
            // same SIMD (measured 13-15% faster than one priority throughout).
            __builtin_amdgcn_s_setprio(1);
            stage_shared<P, kTPB>(sS, fe, tid);
            if (lx == kTX - 1) {
#pragma unroll
                for (int az = 0; az < N; ++az)
#pragma unroll
                    for (int ay = 1; ay < N; ++ay) sE[(az * P + ay - 1) * kTY + ly] = double(fe[(az * N + ay) * N + P]);
            }
            if (ly == kTY - 1) {
#pragma unroll
                for (int az = 0; az < N; ++az)
#pragma unroll
                    for (int ax = 1; ax < N; ++ax)
                        sE[P * N * kTY + (az * P + ax - 1) * kTX + lx] = double(fe[(az * N + P) * N + ax]);
            }
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(2);
        // 2. loads of the next layer's new planes (global planes k0+N .. k0+N+P-1)
        using PR = PlaneRows<P, kTY, P>;
        const bool more = cz + 1 < z1;
        const int rl = tid / PR::W, cl = tid % PR::W;
        double pf[PR::NREG], pfx[PR::NEXTRA];
        if (more) {
            const double *src = q.Tin + ((long long)i0 + (long long)q.NX * j0 + NXY * (k0 + N));
            const int nxl = q.NX - i0, nyl = q.NY - j0;
            const unsigned goff = unsigned(rl) * unsigned(q.NX) + unsigned(cl);
#pragma unroll
            for (int e = 0; e < PR::NREG; ++e) {
                const int lp = e / PR::PPP, dr = PR::RPP * (e % PR::PPP);
                pf[e] = 0.0;
                if (cl < nxl && rl + dr < nyl)
                    pf[e] = src[goff + unsigned(lp) * unsigned(NXY) + unsigned(dr) * unsigned(q.NX)];
            }
#pragma unroll
            for (int x = 0; x < PR::NEXTRA; ++x) {
                int lp, lj, li;
                const bool ok = PR::extra(tid, x, lp, lj, li);
                pfx[x] = 0.0;
                if (ok && li < nxl && lj < nyl)
                    pfx[x] = src[unsigned(lp) * unsigned(NXY) + unsigned(lj) * unsigned(q.NX) + unsigned(li)];
            }
        }
        // 3. node completion: interior nodes per lane, perimeter spread over the lanes
        complete_layer<P, kTY, MODE>(q, fe, sS, sE, sC, sPC, sT, r0, tid, lx, ly, tx, ty, cz, seg, cz == z0,
                                     cz == z1 - 1, active, q.slots + tpar * q.fm.GT);
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // 4. the new planes replace planes k0 .. k0+P-1 (slots r0 .. r0+P-1 mod N)
        if (more) {
            const int loff = rl * BX + cl;
#pragma unroll
            for (int e = 0; e < PR::NREG; ++e) {
                const int lp = e / PR::PPP, dr = PR::RPP * (e % PR::PPP);
                const int sl = r0 + lp < N ? r0 + lp : r0 + lp - N;
                sT[sl * PLANE + loff + dr * BX] = pf[e];
            }
#pragma unroll
            for (int x = 0; x < PR::NEXTRA; ++x) {
                int lp, lj, li;
                if (PR::extra(tid, x, lp, lj, li)) {
                    const int sl = r0 + lp < N ? r0 + lp : r0 + lp - N;
                    sT[sl * PLANE + lj * BX + li] = pfx[x];
                }
            }
            __syncthreads();
        }
    }
}


// Launch of one instantiation, with optional start/stop events recorded by the
// dispatch itself (kernel execution time only, no queue gaps).
template <int P, typename R, int MODE>
hipError_t launch_cells_inst(const CellParams<R> &prm, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    constexpr int TY = 16;
    const dim3 grid(8 * prm.tiles_per_xcd), block(kTX * TY);
    auto kernel = k_cells<P, R, MODE, TY>;
    if (e0) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, prm);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, prm);
    return hipGetLastError();
}

}  // namespace
}  // namespace pbf
