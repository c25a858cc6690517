// Discrete adjoint of the explicit step and the probe objective (gfx950).
//
// The forward step (Section 3.2, eq. forward_euler, with the operator of
// Section 4.2 and the law of Section 2) maps the state (T_n, r^{n-1}) to
//   r^n     = max(r^{n-1}, g(T_n))                     at every powder point,
//   T_{n+1} = T_n + dt f(T_n, r^n) / C~(T_n)           at free nodes.
// Its transpose Jacobian, applied to lambda_{n+1} and the history adjoint mu_n,
// is, with a = dt lambda_{n+1} / C~ (0 at Dirichlet nodes):
//   lambda_n = lambda_{n+1} - a f c'(T)/c(T)          (identity and nodal capacity,
//                                                      free nodes only)
// where a f = lambda_{n+1} (T_{n+1} - T_n) at free nodes, so the forward vector f
// need not be re-assembled: the step's own output gives it.
//            + sum_e G_e^T [ -sum_q W k grad N . grad a_h            (symmetric part)
//                            + sum_q N Tbar_q ],                     (law part)
//   Tbar_q = k_T kbar_q + [g > r^{n-1}] g' rbar_q,  kbar_q = -W grad a_h . grad T_h,
//   rbar_q = k_r kbar_q + mu_q,   mu_q <- [g <= r^{n-1}] rbar_q,
// and the source sensitivity of the step, dJ/dW_track += sum_q W a_h s_q / W,
// for the track the beam is on.  Derivatives of the law are one-sided: the
// slope of the table segment the forward evaluation used (zero outside the
// table), g' on the open melting interval, and no derivative of the
// latent-heat box.
//
// Same column-march structure as the other cell kernels (one wavefront per
// 16 x 4 column, z-carry, owner-computes node sums in a fixed order, parity
// slots for column faces), with T and a staged in LDS.
#include <hip/hip_runtime.h>

#include "cellkit.h"

namespace pbf {
namespace {

constexpr int kATY = 4;

// c'(T) / c(T) at a node: slope of the c_p table on the segment that holds T
// (left-closed, zero outside the open table range) over the apparent capacity
__device__ __forceinline__ double capacity_log_slope(ConstLaw<double> &L, double T)
{
    double c = L.c0, cs = 0.0;
    // unrolled over the table size with a uniform guard, so that the law's
    // coefficients are loaded together instead of one round trip per hinge
#pragma unroll
    for (int i = 0; i < kMaxBp; ++i) {
        if (i >= L.n_hinge) break;
        const double x = T - L.b[i];
        c = __builtin_fma(L.dc[i], fmax0(x, 0.0), c);
        cs += x >= 0.0 ? L.dc[i] : 0.0;
    }
    if (L.n_hinge == 0 || !(T > L.b[0]) || T >= L.b[L.n_hinge - 1]) cs = 0.0;
    if (T >= L.Ts && T <= L.Tl) c += L.lat;
    return cs / c;
}

template <int P>
__global__ void __launch_bounds__(kTX * kATY) __attribute__((amdgpu_waves_per_eu(P == 2 ? 1 : 2)))
k_adjoint(const AdjointParams p)
{
    constexpr int kTY = kATY, kTPB = kTX * kTY;
    constexpr int N = P + 1, NN = N * N * N;
    constexpr int BX = P * kTX + 1, BY = P * kTY + 1, PLANE = BX * BY, NB = N * PLANE;
    constexpr int NSH = N * N + P * N;
    using TB = Tables<P>;
    __shared__ double sT[3][NB];  // T_n, a, node term of lambda_n (below)
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
    double src_acc = 0.0;  // this lane's share of sum_q W a_h s_q / W

#pragma clang loop unroll(disable)
    for (int cz = z0; cz < z1; ++cz) {
        const int k0 = P * cz;
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        AS4<AdjointParams> &q = *kernarg_params<AdjointParams>();
        ConstLaw<double> &law = const_law(q.law);
        const int lx = tid % kTX, ly = tid / kTX;
        const int cx = kTX * tx + lx, cy = kTY * ty + ly;
        const bool active = cx < q.nx && cy < q.ny;
        {
            // all loads of the lane first (their latencies overlap); then, per
            // node of the block, the capacity c(T_n) and its slope (hinge sums one
            // hinge at a time, each coefficient read once), a = dt lambda / C~ and
            // the node term lambda - lambda (T_{n+1} - T_n) c'(T_n) / c(T_n) of
            // lambda_n (zero at Dirichlet nodes)
            constexpr int NL = (NB + kTPB - 1) / kTPB;
            double Tv[NL], lv[NL], t1v[NL];
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                const int idx = tid + e * kTPB;
                const int li = idx % BX, lj = (idx / BX) % BY, lk = idx / PLANE;
                const int gi = i0 + li, gj = j0 + lj, gk = k0 + lk;
                const bool in = idx < NB && gi < q.NX && gj < q.NY;
                const long long g = (long long)gi + (long long)q.NX * gj + NXY * gk;
                Tv[e] = in ? q.T[g] : 0.0;
                lv[e] = in ? q.lam[g] : 0.0;
                t1v[e] = in ? q.Tn1[g] : 0.0;
            }
            double c[NL], cs[NL];
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                c[e] = law.c0;
                cs[e] = 0.0;
            }
            for (int i = 0; i < law.n_hinge; ++i) {
                const double bi = law.b[i], dci = law.dc[i];
#pragma unroll
                for (int e = 0; e < NL; ++e) {
                    const double x = Tv[e] - bi;
                    c[e] = __builtin_fma(dci, fmax0(x, 0.0), c[e]);
                    cs[e] += x >= 0.0 ? dci : 0.0;
                }
            }
            const double b_lo = law.n_hinge > 0 ? double(law.b[0]) : 0.0;
            const double b_hi = law.n_hinge > 0 ? double(law.b[law.n_hinge - 1]) : 0.0;
#pragma unroll
            for (int e = 0; e < NL; ++e) {
                const int idx = tid + e * kTPB;
                if (idx >= NB) continue;
                const int li = idx % BX, lj = (idx / BX) % BY, lk = idx / PLANE;
                const int gi = i0 + li, gj = j0 + lj, gk = k0 + lk;
                const bool in = gi < q.NX && gj < q.NY;
                const double T = Tv[e];
                if (law.n_hinge == 0 || !(T > b_lo) || T >= b_hi) cs[e] = 0.0;
                if (T >= law.Ts && T <= law.Tl) c[e] += law.lat;
                // C~ as in the forward step (nodal capacity)
                const double m = lumped_mass_1d(gi, q.NX, P, q.hx) * lumped_mass_1d(gj, q.NY, P, q.hy) *
                                 lumped_mass_1d(gk, q.NZ, P, q.hz);
                const double C = law.rho * c[e] * m;
                const bool unconstrained = in && !on_dirichlet(q.dmask, gi, gj, gk, q.NX, q.NY, q.NZ);
                const double lam = lv[e];
                sT[0][idx] = T;
                sT[1][idx] = unconstrained ? q.dt * lam / C : 0.0;
                sT[2][idx] = unconstrained ? lam - lam * (t1v[e] - T) * (cs[e] / c[e]) : 0.0;
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
            const long long hc =
                has_hist ? (long long)cx + (long long)q.nx * (cy + (long long)q.ny * (cz - q.hist_cz0)) : 0;
            const bool src_cell = q.src_on && q.laser_kind == 1 && cz >= q.src_cz0;
            double u[NN], t1[NN], t2[NN], vT[NN], va[NN], w[NN];
            gather(0, u);
            sweep<TagS<P>, N, 0>(u, t1);
            sweep<TagS<P>, N, 1>(t1, t2);
            sweep<TagS<P>, N, 2>(t2, vT);
            gather(1, u);
            sweep<TagS<P>, N, 0>(u, t1);
            sweep<TagS<P>, N, 1>(t1, t2);
            sweep<TagS<P>, N, 2>(t2, va);
            // hinges that some Gauss point of the wave reaches (T >= b_i)
            double tmax = vT[0];
#pragma unroll
            for (int a = 1; a < NN; ++a) tmax = fmax0(tmax, vT[a]);
            int nh = 0;
            while (nh < law.n_hinge && __any(tmax >= law.b[nh])) ++nh;
            const double b_first = law.n_hinge > 0 ? double(law.b[0]) : 0.0;
            const double b_last = law.n_hinge > 0 ? double(law.b[law.n_hinge - 1]) : 0.0;
            // hinge sums of every point, one hinge at a time (each coefficient
            // read once per cell; every point adds its hinges in increasing order)
            double kq[NN], ksq[NN];
#pragma unroll
            for (int a = 0; a < NN; ++a) {
                kq[a] = law.k0;
                ksq[a] = 0.0;
            }
            for (int i = 0; i < nh; ++i) {
                const double bi = law.b[i], dki = law.dk[i];
#pragma unroll
                for (int a = 0; a < NN; ++a) {
                    const double x = vT[a] - bi;
                    kq[a] = __builtin_fma(dki, fmax0(x, 0.0), kq[a]);
                    ksq[a] += x >= 0.0 ? dki : 0.0;
                }
            }
            // the Gaussian once per (x, y) column of points (its exponent does not depend on z)
            double sq[N * N];
            if (src_cell) {
                sfor<0, N * N>([&](auto ic) {
                    constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
                    constexpr double xi = TB::gp(i), et = TB::gp(j);
                    const double dxb = (cx + xi) * q.hx - q.xb, dyb = (cy + et) * q.hy - q.yb;
                    sq[decltype(ic)::value] = exp(-(dxb * dxb + dyb * dyb) * q.two_over_R2);
                });
            }
#pragma unroll
            for (int a = 0; a < NN; ++a) w[a] = 0.0;
            // history r and its adjoint mu of a z-plane of points, loaded together
            // before the plane (the mu stores would otherwise order each point's
            // loads behind the previous point's store)
            double rpl[N * N], mul[N * N];
            sfor<0, NN>([&](auto qc) {
                constexpr int qq = decltype(qc)::value;
                constexpr int qx = qq % N, qy = (qq / N) % N, qz = qq / (N * N);
                if constexpr (qx == 0 && qy == 0) {
                    if (has_hist) {
#pragma unroll
                        for (int j = 0; j < N * N; ++j) {
                            const long long hj = (long long)(qz * N * N + j) * q.n_hist_cells + hc;
                            rpl[j] = q.hist[hj];
                            mul[j] = q.mu[hj];
                        }
                    }
                }
                auto tx_ = [&](auto rc) { return vT[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
                auto ty_ = [&](auto rc) { return vT[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
                auto tz_ = [&](auto rc) { return vT[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
                auto ax_ = [&](auto rc) { return va[tidx<N, 0>(decltype(rc)::value, qy, qz)]; };
                auto ay_ = [&](auto rc) { return va[tidx<N, 1>(decltype(rc)::value, qx, qz)]; };
                auto az_ = [&](auto rc) { return va[tidx<N, 2>(decltype(rc)::value, qx, qy)]; };
                const double gTx = rowdot<TagD<P>, qx, 0, N, false>(tx_, 0.0);
                const double gTy = rowdot<TagD<P>, qy, 0, N, false>(ty_, 0.0);
                const double gTz = rowdot<TagD<P>, qz, 0, N, false>(tz_, 0.0);
                const double gax = rowdot<TagD<P>, qx, 0, N, false>(ax_, 0.0);
                const double gay = rowdot<TagD<P>, qy, 0, N, false>(ay_, 0.0);
                const double gaz = rowdot<TagD<P>, qz, 0, N, false>(az_, 0.0);
                const double T = vT[qq];
                const double kpl = kq[qq];
                const double ks = (!(T > b_first) || T >= b_last) ? 0.0 : ksq[qq];
                constexpr double wq = TB::gw(qx) * TB::gw(qy) * TB::gw(qz);
                const double W = wq * q.detJ;
                double rn = 1.0, rp = 1.0, gl = 0.0;
                long long hi = 0;
                if (has_hist) {
                    hi = (long long)qq * q.n_hist_cells + hc;
                    rp = rpl[qy * N + qx];
                    gl = fmin0(fmax0((T - law.Ts) * law.inv_dT, 0.0), 1.0);
                    rn = gl > rp ? gl : rp;
                }
                const double phase = rn + law.phi * (1.0 - rn);
                const double k = has_hist ? kpl * phase : kpl;
                const double kbar = -W * (q.ih2x * gTx * gax + q.ih2y * gTy * gay + q.ih2z * gTz * gaz);
                double Tbar = kbar * (ks * phase);
                if (has_hist) {
                    const double rbar = __builtin_fma(kbar, kpl * (1.0 - law.phi), mul[qy * N + qx]);
                    if (gl > rp) {  // the max took g: the adjoint flows to T
                        const double gp = T < law.Tl ? double(law.inv_dT) : 0.0;
                        Tbar = __builtin_fma(rbar, gp, Tbar);
                        q.mu[hi] = 0.0;
                    } else {
                        q.mu[hi] = rbar;
                    }
                }
                w[qq] += Tbar;
                const double kW = k * W;
                const double Fx = -kW * q.ih2x * gax, Fy = -kW * q.ih2y * gay, Fz = -kW * q.ih2z * gaz;
                sfor<0, N>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    constexpr double dx = TB::D(qx, r), dy = TB::D(qy, r), dz = TB::D(qz, r);
                    if constexpr (dx != 0.0) w[tidx<N, 0>(r, qy, qz)] = __builtin_fma(dx, Fx, w[tidx<N, 0>(r, qy, qz)]);
                    if constexpr (dy != 0.0) w[tidx<N, 1>(r, qx, qz)] = __builtin_fma(dy, Fy, w[tidx<N, 1>(r, qx, qz)]);
                    if constexpr (dz != 0.0) w[tidx<N, 2>(r, qx, qy)] = __builtin_fma(dz, Fz, w[tidx<N, 2>(r, qx, qy)]);
                });
                if (src_cell) {
                    constexpr double ze = TB::gp(qz);
                    const double depth = q.Lz - (cz + ze) * q.hz;
                    if (depth >= 0.0 && depth <= q.h_powder) src_acc += W * va[qq] * q.src_unit * sq[qy * N + qx];
                }
            });
            sweep<TagSt<P>, N, 0>(w, t1);
            sweep<TagSt<P>, N, 1>(t1, t2);
            sweep<TagSt<P>, N, 2>(t2, fe);
            // surface flux on the top face: sum_ij W_ij a_h(x_ij, Lz) s_ij / W
            if (q.src_on && q.laser_kind == 0 && cz == q.nz - 1) {
                gather(1, u);
                sfor<0, N * N>([&](auto ic) {
                    constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
                    constexpr double xi = TB::gp(i), et = TB::gp(j), w2 = TB::gw(i) * TB::gw(j);
                    double ah = 0.0;
                    sfor<0, N * N>([&](auto nc) {
                        constexpr int ax = decltype(nc)::value % N, ay = decltype(nc)::value / N;
                        constexpr double c = TB::S(i, ax) * TB::S(j, ay);
                        if constexpr (c != 0.0) ah = __builtin_fma(c, u[(P * N + ay) * N + ax], ah);
                    });
                    const double dxb = (cx + xi) * q.hx - q.xb, dyb = (cy + et) * q.hy - q.yb;
                    src_acc += w2 * q.hx * q.hy * q.src_unit * exp(-(dxb * dxb + dyb * dyb) * q.two_over_R2) * ah;
                });
            }
            stage_shared<P, kTPB>(sS, fe, tid);
        }
        __syncthreads();
        if (active) {
            owner_nodes<P, kTY>(fe, sS, sC, tid, lx, ly, cx, cy, q.nx, q.ny, k0, seg, cz == z0, cz == z1 - 1,
                                q.NX, q.NY, q.NZ, q.slots + tpar * q.fm.GT, face_map_of(q), NXY,
                                [&](long long g, int gi, int gj, int gk, int ax, int ay, int az, double fs) {
                q.lam_out[g] = sT[2][(az * BY + P * ly + ay) * BX + P * lx + ax] + fs;
            });
        }
        __syncthreads();
    }
    // tile sum of the source sensitivity, fixed butterfly order
    for (int off = 32; off > 0; off >>= 1) src_acc += __shfl_xor(src_acc, off);
    if (threadIdx.x == 0) p.partials[id] = src_acc;
}

__global__ void __launch_bounds__(256) k_adjoint_halo(const AdjointHalo ah)
{
    const HaloParams &h = ah.h;
    FaceNode fn;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!face_node(t, h, fn)) return;
    const long long g = (long long)fn.gi + (long long)h.NX * fn.gj + (long long)h.NX * h.NY * fn.gk;
    const double fs = face_sum(h.slots, h.GX + h.GY + h.GZ, t, fn);
    double base = 0.0;
    if (!on_dirichlet(h.dmask, int(fn.gi), int(fn.gj), int(fn.gk), h.NX, h.NY, h.NZ)) {
        const double lam = ah.lam[g], Tn = h.Tin[g];
        base = lam - lam * (ah.Tn1[g] - Tn) * capacity_log_slope(const_law(h.nlaw), Tn);
    }
    ah.lam_out[g] = base + fs;
}

__device__ __forceinline__ double block_sum_256(double v, double *s)
{
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) s[t] += s[t + w];
        __syncthreads();
    }
    return s[0];
}

__global__ void __launch_bounds__(256) k_adjoint_finish(const double *partials, int n, double *dJdW, int track)
{
    __shared__ double s[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partials[i];
    const double tot = block_sum_256(v, s);
    if (threadIdx.x == 0) dJdW[track] += tot;
}

__global__ void __launch_bounds__(256) k_adjoint_params(const double *dJdW, const double *powers, double A,
                                                        int n, double *dJdP, double *dJdA)
{
    for (int k = threadIdx.x; k < n; k += 256)
        if (dJdP) dJdP[k] = A * dJdW[k];
    if (threadIdx.x == 0 && dJdA) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = __builtin_fma(powers[k], dJdW[k], s);
        dJdA[0] = s;
    }
}

__device__ __forceinline__ long long probe_node(const ProbeSet &ps, int p, int a, double *wgt)
{
    const int N = ps.P + 1;
    const int ax = a % N, ay = (a / N) % N, az = a / (N * N);
    const int *c = ps.cell + 3 * p;
    const double *xi = ps.xi + 3 * p;
    *wgt = lagrange1(ps.P, ax, xi[0]) * lagrange1(ps.P, ay, xi[1]) * lagrange1(ps.P, az, xi[2]);
    return (long long)(ps.P * c[0] + ax) + (long long)ps.NX * (ps.P * c[1] + ay) + ps.NXY * (ps.P * c[2] + az);
}

__device__ __forceinline__ double probe_value(const ProbeSet &ps, int p, const double *T)
{
    const int N = ps.P + 1;
    double v = 0.0;
    for (int a = 0; a < N * N * N; ++a) {
        double wgt;
        const long long g = probe_node(ps, p, a, &wgt);
        v = __builtin_fma(wgt, T[g], v);
    }
    return v;
}

__global__ void __launch_bounds__(256) k_probe_values(const ProbeSet ps, const double *T, double *vals)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < ps.n) vals[p] = probe_value(ps, p, T);
}

constexpr int kMaxProbesDev = 4096;

// J and its gradient with respect to T (lam zeroed beforehand); the scatter
// runs probe by probe so that the sums are reproducible
__global__ void __launch_bounds__(256) k_objective(const ProbeSet ps, const double *T, double *J, double *lam)
{
    __shared__ double e[kMaxProbesDev];
    __shared__ double s[256];
    double v = 0.0;
    for (int p = threadIdx.x; p < ps.n; p += 256) {
        e[p] = probe_value(ps, p, T) - ps.target[p];
        v = __builtin_fma(e[p], e[p], v);
    }
    const double tot = block_sum_256(v, s);
    if (threadIdx.x == 0) J[0] = tot;
    const int NN = (ps.P + 1) * (ps.P + 1) * (ps.P + 1);
    for (int p = 0; p < ps.n; ++p) {
        if ((int)threadIdx.x < NN) {
            double wgt;
            const long long g = probe_node(ps, p, threadIdx.x, &wgt);
            lam[g] += 2.0 * e[p] * wgt;
        }
        __syncthreads();
    }
}

}  // namespace

int adjoint_column_height() { return kATY; }
int adjoint_resident_columns_per_cu() { return 8; }

hipError_t launch_adjoint(int degree, const AdjointParams &ap, const AdjointHalo &ah, hipStream_t s)
{
    const dim3 grid(8 * ap.tiles_per_xcd), block(kTX * kATY);
    if (degree == 1) hipLaunchKernelGGL(k_adjoint<1>, grid, block, 0, s, ap);
    else hipLaunchKernelGGL(k_adjoint<2>, grid, block, 0, s, ap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n = ah.h.GX + ah.h.GY + ah.h.GZ;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_halo, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ah);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish(const double *partials, int ntiles, double *dJdW, int track, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_finish, dim3(1), dim3(256), 0, s, partials, ntiles, dJdW, track);
    return hipGetLastError();
}

hipError_t launch_adjoint_params(const double *dJdW, const double *powers, double A, int n_tracks,
                                 double *dJdP, double *dJdA, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_params, dim3(1), dim3(256), 0, s, dJdW, powers, A, n_tracks, dJdP, dJdA);
    return hipGetLastError();
}

hipError_t launch_probe_values(const ProbeSet &ps, const double *T, double *vals, hipStream_t s)
{
    if (ps.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_values, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps, T, vals);
    return hipGetLastError();
}

hipError_t launch_objective(const ProbeSet &ps, const double *T, double *J, double *lam, long long n,
                            hipStream_t s)
{
    if (ps.n > kMaxProbesDev) return hipErrorInvalidValue;
    hipError_t e = launch_fill(lam, 0.0, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, s, ps, T, J, lam);
    return hipGetLastError();
}

}  // namespace pbf
