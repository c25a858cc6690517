// Kernels of the implicit backward-Euler step (Section 3.2, eqs.
// backward_euler_nonlinear, Newton_1, Newton_2): the symmetric Picard matrix
// A(T^i) = C(T_n)/dt + K(T^i) (Jacobi-preconditioned CG) and the full Newton
// Jacobian A + L (GMRES), all matrix-free (Section 4.2, eq. matrix_free_eval).
// The residual and the diagonal are evaluated once per Picard/Newton iteration:
//   apply:    y = C(Tc) x1 / dt + K(Tk) x2 - s f_vol      (free rows; 0 on Dirichlet rows)
//   diagonal: diag(A(Tk)) with C(Tc), by sum factorization of squared 1D tables
// with C_ab = sum_q w detJ rho c(Tc_q) N_a N_b (consistent, apparent capacity)
// and K_ab = sum_q w detJ k(Tk_q, r_q) grad N_a . grad N_b, the consolidated
// fraction r held at its value from the start of the step.
//
// Same column-march structure as the explicit kernels (one wavefront per
// 16 x 4 column, z-carry, owner-computes node sums in a fixed order, parity
// slots for column faces), with four staged input vectors.  The Krylov applies
// in between read per-point coefficients cached by k_picard_coef (capacity and
// conductivity weights, and for Newton W k_T and the gradient of T^i) and
// stage only x, in 16 x 16 cell columns (k_picard_capply).
#include <hip/hip_runtime.h>

#include "cellkit.h"

namespace pbf {
namespace {

constexpr int kPTY = 4;  // one wavefront per column workgroup

// MODE 0: apply (residual with the source), MODE 1: diagonal
template <int P, int MODE>
__global__ void __launch_bounds__(kTX * kPTY) __attribute__((amdgpu_waves_per_eu(2)))
k_picard(const PicardParams p)
{
    constexpr int kTY = kPTY, kTPB = kTX * kTY;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY, NB = N * PLANE;
    constexpr int NSH = N * N + P * N;
    constexpr int NV = MODE == 0 ? 4 : 2;  // staged vectors: Tc, Tk (, x1, x2)
    using TB = Tables<P>;
    __shared__ double sT[NV][NB];
    __shared__ double sS[NSH * kTPB];
    __shared__ double sC[N * N * kTPB];

    const int b = blockIdx.x;
    const int id = (b & 7) * p.tiles_per_xcd + (b >> 3);
    if (id >= p.ntiles) return;
    const int seg = id % p.MZ, col = id / p.MZ;
    const int tx = col % p.MX, ty = col / p.MX;
    const int z0 = p.zb[seg], z1 = p.zb[seg + 1];
    const int i0 = P * kTX * tx, j0 = P * kTY * ty;
    const int tpar = (tx & 1) | ((ty & 1) << 1) | ((seg & 1) << 2);
    const long long NXY = (long long)p.NX * p.NY;

#pragma clang loop unroll(disable)
    for (int cz = z0; cz < z1; ++cz) {
        const int k0 = P * cz;
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        AS4<PicardParams> &q = *kernarg_params<PicardParams>();
        ConstLaw<double> &law = const_law(q.law);
        const int lx = tid % kTX, ly = tid / kTX;
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool active = cx < q.nx && cy < q.ny;
        {
            // all loads of the lane first, so that their latencies overlap
            constexpr int NL = (NB + kTPB - 1) / kTPB, NV = MODE == 0 ? 4 : 2;
            double bv[NV][NL];
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                const int idx = tid + e * kTPB;
                const int li = idx % BX, lj = (idx / BX) % BY, lk = idx / PLANE;
                const int gi = i0 + li, gj = j0 + lj;
                const bool in = idx < NB && gi < q.NX && gj < q.NY;
                const long long g = (long long)gi + (long long)q.NX * gj + NXY * (k0 + lk);
                bv[0][e] = in ? q.Tc[g] : 0.0;
                bv[1][e] = in ? q.Tk[g] : 0.0;
                if constexpr (MODE == 0) {
                    bv[2][e] = in ? q.x1[g] : 0.0;
                    bv[3][e] = in ? q.x2[g] : 0.0;
                }
            }
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                const int idx = tid + e * kTPB;
                if (idx >= NB) continue;
#pragma unroll
                for (int v = 0; v < NV; ++v) sT[v][idx] = bv[v][e];
            }
        }
        __syncthreads();
        auto gather = [&](int vec, double *u) {
#pragma unroll
            for (int a = 0; a < NN; ++a) {
                const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
                u[a] = sT[vec][(az * BY + P * ly + ay) * BX + P * lx + ax];
            }
        };
        double fe[NN];
        if (active) {
            const bool has_hist = cz >= q.hist_cz0;
            const long long hc = has_hist ? (long long)cx + (long long)q.nx * (cy + (long long)q.ny * (cz - q.hist_cz0)) : 0;
            double u[NN], t1[NN], t2[NN], m[NN], kw[NN];
            // capacity weights rho c(Tc_q) W / dt
            gather(0, u);
            sweep<TagS<P>, N, 0>(u, t1);
            sweep<TagS<P>, N, 1>(t1, t2);
            sweep<TagS<P>, N, 2>(t2, m);
            sfor<0, NN>([&](auto qc) {
                constexpr int qq = decltype(qc)::value;
                constexpr double wq = TB::gw(qq % N) * TB::gw((qq / N) % N) * TB::gw(qq / (N * N));
                m[qq] = wq * q.detJ * law.rho * law_c(law, m[qq]) * q.inv_dt;
            });
            // conductivity weights k(Tk_q, r_q) W
            gather(1, u);
            sweep<TagS<P>, N, 0>(u, t1);
            sweep<TagS<P>, N, 1>(t1, t2);
            sweep<TagS<P>, N, 2>(t2, kw);
            sfor<0, NN>([&](auto qc) {
                constexpr int qq = decltype(qc)::value;
                constexpr double wq = TB::gw(qq % N) * TB::gw((qq / N) % N) * TB::gw(qq / (N * N));
                const double r = has_hist ? q.hist[(long long)qq * q.n_hist_cells + hc] : 1.0;
                kw[qq] = wq * q.detJ * law_k(law, kw[qq], r);
            });
            if constexpr (MODE == 0) {
                // mass part: m_q * x1_q, minus the source, as the value integrand
                gather(2, u);
                sweep<TagS<P>, N, 0>(u, t1);
                sweep<TagS<P>, N, 1>(t1, t2);
                sweep<TagS<P>, N, 2>(t2, u);
#pragma unroll
                for (int a = 0; a < NN; ++a) m[a] *= u[a];
                if (q.src_on && q.laser_kind == 1 && cz >= q.src_cz0) {
                    sfor<0, NN>([&](auto qc) {
                        constexpr int qq = decltype(qc)::value;
                        constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
                        constexpr double xi = TB::gp(qx), et = TB::gp(qy), ze = TB::gp(qz);
                        constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
                        const double depth = q.Lz - (cz + ze) * q.hz;
                        if (depth >= 0.0 && depth <= q.h_powder) {
                            const double dxb = (cx + xi) * q.hx - q.xb, dyb = (cy + et) * q.hy - q.yb;
                            m[qq] -= wq * q.detJ * q.src_amp * exp(-(dxb * dxb + dyb * dyb) * q.two_over_R2);
                        }
                    });
                }
                // diffusion part: + D^T (k W h^-2 grad x2) in collocation space
                gather(3, u);
                sweep<TagS<P>, N, 0>(u, t1);
                sweep<TagS<P>, N, 1>(t1, t2);
                sweep<TagS<P>, N, 2>(t2, u);
                sfor<0, NN>([&](auto qc) {
                    constexpr int qq = decltype(qc)::value;
                    constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
                    auto gxf = [&](auto rc) { return u[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
                    auto gyf = [&](auto rc) { return u[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
                    auto gzf = [&](auto rc) { return u[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
                    const double Fx = kw[qq] * q.ih2x * rowdot<TagD<P>, qx, 0, N, false>(gxf, 0.0);
                    const double Fy = kw[qq] * q.ih2y * rowdot<TagD<P>, qy, 0, N, false>(gyf, 0.0);
                    const double Fz = kw[qq] * q.ih2z * rowdot<TagD<P>, qz, 0, N, false>(gzf, 0.0);
                    sfor<0, N>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
                        if constexpr (dx != 0.0) m[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, m[tidx<N, 0>(r, qy, qz)]);
                        if constexpr (dy != 0.0) m[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, m[tidx<N, 1>(r, qx, qz)]);
                        if constexpr (dz != 0.0) m[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, m[tidx<N, 2>(r, qx, qy)]);
                    });
                });
                integrate3<TagSt<P>, TagSt<P>, TagSt<P>, N>(m, fe);
                // Gaussian surface flux on the top face, subtracted like the volume source
                if (q.src_on && q.laser_kind == 0 && cz == q.nz - 1) {
                    sfor<0, N>([&](auto ac) {
                        constexpr int ax = decltype(ac)::value;
                        sfor<0, N>([&](auto bc) {
                            constexpr int ay = decltype(bc)::value;
                            double s = 0.0;
                            sfor<0, N * N>([&](auto ic) {
                                constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
                                constexpr double c = TB::S(i, ax) * TB::S(j, ay) * TB::gw(i) * TB::gw(j);
                                constexpr double xi = TB::gp(i), et = TB::gp(j);
                                if constexpr (c != 0.0) {
                                    const double dxb = (cx + xi) * q.hx - q.xb, dyb = (cy + et) * q.hy - q.yb;
                                    s += c * q.hx * q.hy * q.src_amp * exp(-(dxb * dxb + dyb * dyb) * q.two_over_R2);
                                }
                            });
                            fe[(P * N + ay) * N + ax] -= s;
                        });
                    });
                }
            } else {
                // diag = (S2 S2 S2)^T m + sum_d h_d^-2 (S2 .. Dn2 in d .. S2)^T kW
                double acc[NN];
                integrate3<TagS2t<P>, TagS2t<P>, TagS2t<P>, N>(m, fe);
                integrate3<TagDn2t<P>, TagS2t<P>, TagS2t<P>, N>(kw, acc);
#pragma unroll
                for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(q.ih2x, acc[a], fe[a]);
                integrate3<TagS2t<P>, TagDn2t<P>, TagS2t<P>, N>(kw, acc);
#pragma unroll
                for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(q.ih2y, acc[a], fe[a]);
                integrate3<TagS2t<P>, TagS2t<P>, TagDn2t<P>, N>(kw, acc);
#pragma unroll
                for (int a = 0; a < NN; ++a) fe[a] = __builtin_fma(q.ih2z, acc[a], fe[a]);
            }
            stage_shared<P, kTPB>(sS, fe, tid);
        }
        __syncthreads();
        if (active) {
            owner_nodes<P, kTY>(fe, sS, sC, tid, lx, ly, cx, cy, q.nx, q.ny, k0, seg, cz == z0, cz == z1 - 1,
                                q.NX, q.NY, q.NZ, q.slots + tpar * q.fm.GT, face_map_of(q), NXY,
                                [&](long long g, int gi, int gj, int gk, int, int, int, double f) {
                const bool dir = on_dirichlet(q.dmask, gi, gj, gk, q.NX, q.NY, q.NZ);
                q.yout[g] = dir ? (MODE == 0 ? 0.0 : 1.0) : f;
            });
        }
        __syncthreads();
    }
}

// Per-point coefficients of the Krylov applies, one thread per cell (cells in
// x-fastest order, so point-major stores are coalesced): the arithmetic of the
// capacity and conductivity weights (and of the Newton term) is that of
// k_picard, so applies from the cache equal k_picard's applies bit for bit.
template <int P, bool NEWTON>
__global__ void __launch_bounds__(256) k_picard_coef(const PicardParams p)
{
    using TB = Tables<P>;
    constexpr int N = P + 1, NN = N * N * N;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= p.ncells) return;
    ConstLaw<double> &law = const_law(p.law);
    const int cx = int(c % p.nx), cy = int((c / p.nx) % p.ny), cz = int(c / ((long long)p.nx * p.ny));
    const long long NXY = (long long)p.NX * p.NY;
    const bool has_hist = cz >= p.hist_cz0;
    const long long hc = has_hist ? (long long)cx + (long long)p.nx * (cy + (long long)p.ny * (cz - p.hist_cz0)) : 0;
    double u[NN], t1[NN], t2[NN], v[NN];
    auto gather = [&](const double *X) {
#pragma unroll
        for (int a = 0; a < NN; ++a) {
            const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
            u[a] = X[(long long)(P * cx + ax) + (long long)p.NX * (P * cy + ay) + NXY * (P * cz + az)];
        }
    };
    gather(p.Tc);
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, v);
    sfor<0, NN>([&](auto qc) {
        constexpr int qq = decltype(qc)::value;
        constexpr double wq = TB::gw(qq % N) * TB::gw((qq / N) % N) * TB::gw(qq / (N * N));
        p.coef[(long long)qq * p.ncells + c] = wq * p.detJ * law.rho * law_c(law, v[qq]) * p.inv_dt;
    });
    gather(p.Tk);
    sweep<TagS<P>, N, 0>(u, t1);
    sweep<TagS<P>, N, 1>(t1, t2);
    sweep<TagS<P>, N, 2>(t2, v);
    sfor<0, NN>([&](auto qc) {
        constexpr int qq = decltype(qc)::value;
        constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
        constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
        const double r = has_hist ? p.hist[(long long)qq * p.n_hist_cells + hc] : 1.0;
        p.coef[(long long)(NN + qq) * p.ncells + c] = wq * p.detJ * law_k(law, v[qq], r);
        if constexpr (NEWTON) {
            auto gxf = [&](auto rc) { return v[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
            auto gyf = [&](auto rc) { return v[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
            auto gzf = [&](auto rc) { return v[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
            p.coef[(long long)(2 * NN + qq) * p.ncells + c] = wq * p.detJ * law_kT(law, v[qq], r);
            p.coef[(long long)(3 * NN + qq) * p.ncells + c] = rowdot<TagD<P>, qx, 0, N, false>(gxf, 0.0);
            p.coef[(long long)(4 * NN + qq) * p.ncells + c] = rowdot<TagD<P>, qy, 0, N, false>(gyf, 0.0);
            p.coef[(long long)(5 * NN + qq) * p.ncells + c] = rowdot<TagD<P>, qz, 0, N, false>(gzf, 0.0);
        }
    });
}

// Krylov apply from the coefficient cache: y = C x/dt + K x (+ L x), free rows;
// 0 on Dirichlet rows.  Column march of 16 x 16 cells with one staged vector.
template <int P, bool NEWTON>
__global__ void __launch_bounds__(kTX * 16) __attribute__((amdgpu_waves_per_eu(2)))
k_picard_capply(const PicardParams p)
{
    constexpr int kTY = 16, kTPB = kTX * kTY;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY, NB = N * PLANE;
    constexpr int NSH = N * N + P * N;
    using TB = Tables<P>;
    __shared__ double sT[NB];
    __shared__ double sS[NSH * kTPB];
    __shared__ double sC[N * N * kTPB];

    const int b = blockIdx.x;
    const int id = (b & 7) * p.tiles_per_xcd + (b >> 3);
    if (id >= p.ntiles) return;
    const int seg = id % p.MZ, col = id / p.MZ;
    const int tx = col % p.MX, ty = col / p.MX;
    const int z0 = p.zb[seg], z1 = p.zb[seg + 1];
    const int i0 = P * kTX * tx, j0 = P * kTY * ty;
    const int tpar = (tx & 1) | ((ty & 1) << 1) | ((seg & 1) << 2);
    const long long NXY = (long long)p.NX * p.NY;

#pragma clang loop unroll(disable)
    for (int cz = z0; cz < z1; ++cz) {
        const int k0 = P * cz;
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        AS4<PicardParams> &q = *kernarg_params<PicardParams>();
        const int lx = tid % kTX, ly = tid / kTX;
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool active = cx < q.nx && cy < q.ny;
        // the cell's conductivity weights, in flight with the block load below
        const long long cell = (long long)cx + (long long)q.nx * (cy + (long long)q.ny * cz);
        const double *cf = q.coef + cell;
        const long long nc = q.ncells;
        double kwq[NN];
#pragma unroll
        for (int a = 0; a < NN; ++a) kwq[a] = active ? cf[(long long)(NN + a) * nc] : 0.0;
        {
            // all loads of the lane first, so that their latencies overlap
            constexpr int NL = (NB + kTPB - 1) / kTPB;
            double xv[NL];
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                const int idx = tid + e * kTPB;
                const int li = idx % BX, lj = (idx / BX) % BY, lk = idx / PLANE;
                const int gi = i0 + li, gj = j0 + lj;
                xv[e] = (idx < NB && gi < q.NX && gj < q.NY)
                            ? q.x2[(long long)gi + (long long)q.NX * gj + NXY * (k0 + lk)] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < NL; ++e)
                if (tid + e * kTPB < NB) sT[tid + e * kTPB] = xv[e];
        }
        __syncthreads();
        double fe[NN];
        if (active) {
            double u[NN], t1[NN], t2[NN], m[NN];
#pragma unroll
            for (int a = 0; a < NN; ++a) m[a] = cf[(long long)a * nc];  // capacity weights, before the sweeps
#pragma unroll
            for (int a = 0; a < NN; ++a) {
                const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
                u[a] = sT[(az * BY + P * ly + ay) * BX + P * lx + ax];
            }
            sweep<TagS<P>, N, 0>(u, t1);
            sweep<TagS<P>, N, 1>(t1, t2);
            sweep<TagS<P>, N, 2>(t2, u);
#pragma unroll
            for (int a = 0; a < NN; ++a) m[a] = m[a] * u[a];
            sfor<0, NN>([&](auto qc) {
                constexpr int qq = decltype(qc)::value;
                constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
                const double kw = kwq[qq];
                auto gxf = [&](auto rc) { return u[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
                auto gyf = [&](auto rc) { return u[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
                auto gzf = [&](auto rc) { return u[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
                const double Fx = kw * q.ih2x * rowdot<TagD<P>, qx, 0, N, false>(gxf, 0.0);
                const double Fy = kw * q.ih2y * rowdot<TagD<P>, qy, 0, N, false>(gyf, 0.0);
                const double Fz = kw * q.ih2z * rowdot<TagD<P>, qz, 0, N, false>(gzf, 0.0);
                sfor<0, N>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
                    if constexpr (dx != 0.0) m[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, m[tidx<N, 0>(r, qy, qz)]);
                    if constexpr (dy != 0.0) m[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, m[tidx<N, 1>(r, qx, qz)]);
                    if constexpr (dz != 0.0) m[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, m[tidx<N, 2>(r, qx, qy)]);
                });
            });
            if constexpr (NEWTON) {
                // the Newton coefficients of a z-plane of points, loaded together
                double nk[N * N], ngx[N * N], ngy[N * N], ngz[N * N];
                sfor<0, NN>([&](auto qc) {
                    constexpr int qq = decltype(qc)::value;
                    constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
                    if constexpr (qx == 0 && qy == 0) {
#pragma unroll
                        for (int j = 0; j < N * N; ++j) {
                            const long long o = (long long)(qz * N * N + j) * nc;
                            nk[j] = cf[2 * NN * nc + o];
                            ngx[j] = cf[3 * NN * nc + o];
                            ngy[j] = cf[4 * NN * nc + o];
                            ngz[j] = cf[5 * NN * nc + o];
                        }
                    }
                    constexpr int j = qy * N + qx;
                    const double kd = nk[j] * u[qq];
                    const double Fx = kd * q.ih2x * ngx[j];
                    const double Fy = kd * q.ih2y * ngy[j];
                    const double Fz = kd * q.ih2z * ngz[j];
                    sfor<0, N>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
                        if constexpr (dx != 0.0) m[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, m[tidx<N, 0>(r, qy, qz)]);
                        if constexpr (dy != 0.0) m[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, m[tidx<N, 1>(r, qx, qz)]);
                        if constexpr (dz != 0.0) m[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, m[tidx<N, 2>(r, qx, qy)]);
                    });
                });
            }
            integrate3<TagSt<P>, TagSt<P>, TagSt<P>, N>(m, fe);
            // staging and node completion at a raised wave priority (short,
            // latency-bound LDS and memory chains; they issue ahead of the
            // other workgroup's cell arithmetic on the same SIMD)
            __builtin_amdgcn_s_setprio(2);
            stage_shared<P, kTPB>(sS, fe, tid);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(2);
        if (active) {
            owner_nodes<P, kTY>(fe, sS, sC, tid, lx, ly, cx, cy, q.nx, q.ny, k0, seg, cz == z0, cz == z1 - 1,
                                q.NX, q.NY, q.NZ, q.slots + tpar * q.fm.GT, face_map_of(q), NXY,
                                [&](long long g, int gi, int gj, int gk, int, int, int, double f) {
                q.yout[g] = on_dirichlet(q.dmask, gi, gj, gk, q.NX, q.NY, q.NZ) ? 0.0 : f;
            });
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_picard_halo(const HaloParams h, double *y)
{
    FaceNode fn;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!face_node(t, h, fn)) return;
    const long long g = (long long)fn.gi + (long long)h.NX * fn.gj + (long long)h.NX * h.NY * fn.gk;
    const double f = face_sum(h.slots, h.GX + h.GY + h.GZ, t, fn);
    const bool dir = on_dirichlet(h.dmask, int(fn.gi), int(fn.gj), int(fn.gk), h.NX, h.NY, h.NZ);
    y[g] = dir ? (MODE == 0 ? 0.0 : 1.0) : f;
}

}  // namespace

int picard_column_height() { return kPTY; }

hipError_t launch_picard_coef(int degree, bool newton, const PicardParams &pp, hipStream_t s)
{
    const dim3 grid((unsigned)((pp.ncells + 255) / 256)), block(256);
    if (degree == 1) {
        if (newton) hipLaunchKernelGGL((k_picard_coef<1, true>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard_coef<1, false>), grid, block, 0, s, pp);
    } else {
        if (newton) hipLaunchKernelGGL((k_picard_coef<2, true>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard_coef<2, false>), grid, block, 0, s, pp);
    }
    return hipGetLastError();
}

hipError_t launch_picard_capply(int degree, bool newton, const PicardParams &pp, const HaloParams &hp,
                                hipStream_t s)
{
    const dim3 grid(8 * pp.tiles_per_xcd), block(kTX * 16);
    if (degree == 1) {
        if (newton) hipLaunchKernelGGL((k_picard_capply<1, true>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard_capply<1, false>), grid, block, 0, s, pp);
    } else {
        if (newton) hipLaunchKernelGGL((k_picard_capply<2, true>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard_capply<2, false>), grid, block, 0, s, pp);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n = hp.GX + hp.GY + hp.GZ;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_picard_halo<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, hp, pp.yout);
    return hipGetLastError();
}

hipError_t launch_picard(int degree, int mode, const PicardParams &pp, const HaloParams &hp,
                         hipStream_t s)
{
    const dim3 grid(8 * pp.tiles_per_xcd), block(kTX * kPTY);
    if (degree == 1) {
        if (mode == 0) hipLaunchKernelGGL((k_picard<1, 0>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard<1, 1>), grid, block, 0, s, pp);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_picard<2, 0>), grid, block, 0, s, pp);
        else hipLaunchKernelGGL((k_picard<2, 1>), grid, block, 0, s, pp);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n = hp.GX + hp.GY + hp.GZ;
    if (n == 0) return hipSuccess;
    const dim3 g2((unsigned)((n + 255) / 256)), b2(256);
    if (mode == 0) hipLaunchKernelGGL(k_picard_halo<0>, g2, b2, 0, s, hp, pp.yout);
    else hipLaunchKernelGGL(k_picard_halo<1>, g2, b2, 0, s, hp, pp.yout);
    return hipGetLastError();
}

}  // namespace pbf
