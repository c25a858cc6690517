// Device building blocks shared by the cell kernels of the pbftherm library:
// compile-time 1D contractions, scalar access to the material law and to the
// kernel arguments, the lumped nodal capacity, and the owner-computes node
// completion of the column-march kernels.  Internal header (device code).
#pragma once

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

// max/min of finite values (one v_max/v_min instruction; the sign of a zero
// result never matters where these are used)
template <typename R> __device__ __forceinline__ R fmax0(R a, R b) { return fmax(a, b); }
template <typename R> __device__ __forceinline__ R fmin0(R a, R b) { return fmin(a, b); }

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

__device__ __forceinline__ bool on_dirichlet(unsigned m, int i, int j, int k, int NX, int NY, int NZ)
{
    return ((m & 1u) && i == 0) || ((m & 2u) && i == NX - 1) || ((m & 4u) && j == 0) ||
           ((m & 8u) && j == NY - 1) || ((m & 16u) && k == 0) || ((m & 32u) && k == NZ - 1);
}

__device__ __forceinline__ bool is_face(int g, int S, int n)  // interior tile face
{
    return g > 0 && g < n - 1 && (g % S) == 0;
}

// Copy of the face map of a parameter block (which may live in the kernel
// argument segment).
template <typename Q>
__device__ __forceinline__ FaceMap face_map_of(Q &q)
{
    return FaceMap{q.fm.GX, q.fm.GY, q.fm.GT};
}

// Index of a column-face node in the compact slot layout: x-face planes
// [plane][k][j], then y-face planes [plane][k][i] (nodes not on an x face),
// then interior z-segment ends [end][j][i] (nodes on neither; zf: the end's
// index, segment s ending at zf = s).  SX, SY: node planes per column in x, y.
__device__ __forceinline__ long long face_slot(int gi, int gj, int gk, int zf, int SX, int SY, int NX,
                                               int NY, int NZ, FaceMap m)
{
    if (is_face(gi, SX, NX)) return ((long long)(gi / SX - 1) * NZ + gk) * NY + gj;
    if (is_face(gj, SY, NY)) return m.GX + ((long long)(gj / SY - 1) * NZ + gk) * NX + gi;
    return m.GX + m.GY + ((long long)zf * NY + gj) * NX + gi;
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


// Outward heat flux density through the free surface at temperature T
// (radiation plus evaporation, see SurfaceLoss); the specific heat of the
// enthalpy term is the law's c_p at [T] (all hinges).
template <typename S>
__device__ __forceinline__ double surface_loss(S &s, double T)
{
    const double T2 = T * T;
    double q = s.eps_sigma * (T2 * T2 - s.Tinf4);
    if (s.evap) {
        const double Tc = fmin(T, s.Tmax);
        if (Tc > s.Tv) {
            ConstLaw<double> &L = const_law(s.law);
            double c = L.c0;
            for (int h = 0; h < L.n_hinge; ++h) c = __builtin_fma(L.dc[h], fmax(Tc - L.b[h], 0.0), c);
            const double mdot = s.CP82 * exp(-s.CT * (1.0 / Tc - s.inv_Tv)) * sqrt(s.CM / Tc);
            q += mdot * (s.hv + c * (Tc - s.Th0));
        }
    }
    return q;
}

// Surface losses of a cell with a face on z = Lz: fe[top node layer] -=
// S^T (w_i w_j hx hy q(T_ij)), T_ij interpolated at the face Gauss points from
// the top node layer values Ttop(ax, ay) (Section 2, eq. bc_rad_evap, weak form).
template <int P, typename S, typename F, typename R>
__device__ __forceinline__ void surface_loss_face(S &s, double hx, double hy, F &&Ttop, R *fe)
{
    using TB = Tables<P>;
    constexpr int N = P + 1;
    double qs[N * N];
    sfor<0, N * N>([&](auto ic) {
        constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
        double Ts = 0.0;
        sfor<0, N * N>([&](auto nc) {
            constexpr int ax = decltype(nc)::value % N, ay = decltype(nc)::value / N;
            constexpr double cc = TB::S(i, ax) * TB::S(j, ay);
            if constexpr (cc != 0.0) Ts = __builtin_fma(cc, Ttop(ax, ay), Ts);
        });
        constexpr double w2 = TB::gw(i) * TB::gw(j);
        qs[decltype(ic)::value] = w2 * hx * hy * surface_loss(s, Ts);
    });
    sfor<0, N * N>([&](auto nc) {
        constexpr int ax = decltype(nc)::value % N, ay = decltype(nc)::value / N;
        double acc = 0.0;
        sfor<0, N * N>([&](auto ic) {
            constexpr int i = decltype(ic)::value % N, j = decltype(ic)::value / N;
            constexpr double cc = TB::S(i, ax) * TB::S(j, ay);
            if constexpr (cc != 0.0) acc = __builtin_fma(cc, qs[decltype(ic)::value], acc);
        });
        fe[(P * N + ay) * N + ax] -= R(acc);
    });
}

// Stage the contributions of a cell that neighbours need: its x = 0 node plane
// and its y = 0 node row (x = 1..P), NSH = (P+1)^2 + P (P+1) values per lane.
template <int P, int kTPB, typename R>
__device__ __forceinline__ void stage_shared(double *sS, const R *fe, int tid)
{
    constexpr int N = P + 1;
#pragma unroll
    for (int az = 0; az < N; ++az) {
#pragma unroll
        for (int ay = 0; ay < N; ++ay) sS[(az * N + ay) * kTPB + tid] = double(fe[(az * N + ay) * N]);
#pragma unroll
        for (int ax = 1; ax <= P; ++ax) sS[(N * N + az * P + ax - 1) * kTPB + tid] = double(fe[az * N * N + ax]);
    }
}

// Owner-computes completion of the nodes of one cell layer in a column.  The
// lane of cell (lx, ly) owns the nodes of its cell with local x and y in 1..P
// (plus 0 on the column's low faces).  The sum order of every node is fixed:
// carry (cells below), own, right, upper, diagonal neighbour.  Top-plane sums
// are carried in sC to the next layer; nodes on column faces and segment ends
// go to the compact slot array `slots` (already offset by the column parity); complete
// nodes are handed to done(g, gi, gj, gk, ax, ay, az, f).
template <int P, int kTY, typename R, typename Done>
__device__ __forceinline__ void owner_nodes(const R *fe, const double *sS, double *sC, int tid, int lx,
                                            int ly, int cx, int cy, int nx, int ny, int k0, int seg,
                                            bool first, bool last, int NX, int NY, int NZ, double *slots,
                                            FaceMap fm, long long NXY, Done &&done)
{
    constexpr int N = P + 1, kTPB = kTX * kTY;
    const bool hasR = lx < kTX - 1 && cx + 1 < nx;
    const bool hasU = ly < kTY - 1 && cy + 1 < ny;
    // nodes with local y = 0 belong to the lanes of the column's first row only
    // (all in the first wavefront): the other wavefronts skip them as a whole
    const bool has_row0 = __builtin_amdgcn_readfirstlane(tid) < kTX;
#pragma unroll
    for (int az = 0; az < N; ++az) {
#pragma unroll
        for (int ay = 0; ay < N; ++ay) {
            if (ay == 0 && !has_row0) continue;  // uniform
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
                const long long g = (long long)gi + (long long)NX * gj + NXY * gk;
                const bool face = (az == 0 && first && gk > 0) || (az == P && last && gk < NZ - 1) ||
                                  is_face(gi, P * kTX, NX) || is_face(gj, P * kTY, NY);
                if (face) {
                    slots[face_slot(gi, gj, gk, az == 0 ? seg - 1 : seg, P * kTX, P * kTY, NX, NY, NZ, fm)] = f;
                    continue;
                }
                done(g, gi, gj, gk, ax, ay, az, f);
            }
        }
    }
}

// Quotient and remainder of n / f.d (see FastDiv).
__device__ __forceinline__ unsigned div_rem(unsigned n, FastDiv f, unsigned &r)
{
    unsigned q = __umulhi(n, f.m);
    r = n - q * f.d;
    if (r >= f.d) {
        ++q;
        r -= f.d;
    }
    return q;
}

// A column-face node and the columns/segments that contain it: cx x cy x cz of
// them (1 or 2 per direction) starting at the tile (x0, y0, z0) whose parity
// bits are p0; the others follow with the parity bit of their direction flipped.
struct FaceNode {
    unsigned gi, gj, gk;
    unsigned p0, cx, cy, cz;
};

// Decode the index t of a column-face node (x-faces, then y-faces without
// x-face nodes, then z segment ends without either; the compact slot order).
// Returns false for threads without a node.
__device__ __forceinline__ bool face_node(unsigned t, const HaloParams &h, FaceNode &fn)
{
    unsigned r = t, gi, gj, gk, plane;
    int grp;
    if (r < unsigned(h.GX)) {
        grp = 0;
        plane = div_rem(div_rem(r, h.fNY, gj), h.fNZ, gk);
        gi = (plane + 1) * unsigned(h.SX);
    } else if ((r -= unsigned(h.GX)) < unsigned(h.GY)) {
        grp = 1;
        plane = div_rem(div_rem(r, h.fNX, gi), h.fNZ, gk);
        gj = (plane + 1) * unsigned(h.SY);
    } else if ((r -= unsigned(h.GY)) < unsigned(h.GZ)) {
        grp = 2;
        plane = div_rem(div_rem(r, h.fNX, gi), h.fNY, gj);
        gk = 0;
        for (int b = 1; b < h.MZ; ++b) gk = plane + 1 == unsigned(b) ? unsigned(h.P * h.zb[b]) : gk;
    } else {
        return false;
    }
    unsigned rx, ry;
    const unsigned tx = div_rem(gi, h.fSX, rx), ty = div_rem(gj, h.fSY, ry);
    const bool fx = rx == 0 && gi > 0 && gi < unsigned(h.NX - 1);
    const bool fy = ry == 0 && gj > 0 && gj < unsigned(h.NY - 1);
    // z: interior segment ends below the node plane, and whether it is one
    unsigned below = 0;
    bool fz = false;
    for (int b = 1; b < h.MZ; ++b) {
        const unsigned e = unsigned(h.P * h.zb[b]);
        below += e < gk ? 1u : 0u;
        fz = fz || e == gk;
    }
    if (grp == 0 && !fx) return false;
    if (grp >= 1 && fx) return false;
    if (grp == 1 && !fy) return false;
    if (grp == 2 && (fy || !fz)) return false;
    // lowest containing tile per direction (the last tile also holds the far boundary)
    const unsigned x0 = fx ? tx - 1 : min(tx, unsigned(h.MX - 1));
    const unsigned y0 = fy ? ty - 1 : min(ty, unsigned(h.MY - 1));
    const unsigned z0 = below;
    fn.gi = gi;
    fn.gj = gj;
    fn.gk = gk;
    fn.p0 = (x0 & 1) | ((y0 & 1) << 1) | ((z0 & 1) << 2);
    fn.cx = fx ? 2 : 1;
    fn.cy = fy ? 2 : 1;
    fn.cz = fz ? 2 : 1;
    return true;
}

// Sum of the parity slots of face node t in a fixed order (z outer, x inner).
__device__ __forceinline__ double face_sum(const double *slots, long long GT, unsigned t, const FaceNode &fn)
{
    double f = 0.0;
    for (unsigned a = 0; a < fn.cz; ++a)
        for (unsigned b = 0; b < fn.cy; ++b)
            for (unsigned e = 0; e < fn.cx; ++e)
                f += slots[(long long)(fn.p0 ^ (e | (b << 1) | (a << 2))) * GT + t];
    return f;
}

// ---- Picard operator helpers (implicit step) ----

template <int P>
struct Dn {  // nodal basis derivative at the Gauss points: l_a'(x_q) = sum_r D(q,r) S(r,a)
    static constexpr double v(int q, int a)
    {
        double s = 0.0;
        for (int r = 0; r <= P; ++r) s += Tables<P>::D(q, r) * Tables<P>::S(r, a);
        return s;
    }
};
template <int P> struct TagS2t  { static constexpr double c(int o, int i) { return Tables<P>::S(i, o) * Tables<P>::S(i, o); } };
template <int P> struct TagDn2t { static constexpr double c(int o, int i) { return Dn<P>::v(i, o) * Dn<P>::v(i, o); } };

// y = S^T-integration of pointwise data in a compact form: out = M3^T M2^T M1^T in
template <class MX, class MY, class MZ, int N>
__device__ __forceinline__ void integrate3(const double *in, double *out)
{
    double t1[N * N * N], t2[N * N * N];
    sweep<MX, N, 0>(in, t1);
    sweep<MY, N, 1>(t1, t2);
    sweep<MZ, N, 2>(t2, out);
}

// conductivity at a Gauss point with the lagged consolidated fraction
// (The hinge loops below are unrolled over the table size with a uniform exit,
// so that the law's coefficients are loaded together rather than one scalar
// round trip per hinge; the sums keep the increasing hinge order.)
template <typename L>
__device__ __forceinline__ double law_k(L &law, double T, double r)
{
    double kpl = law.k0;
#pragma unroll
    for (int i = 0; i < kMaxBp; ++i) {
        if (i >= law.n_hinge) break;
        kpl = __builtin_fma(law.dk[i], fmax0(T - law.b[i], 0.0), kpl);
    }
    return kpl * (r + law.phi * (1.0 - r));
}

// d k / d T at fixed consolidated fraction r: the slope of the table segment
// containing T (right-continuous at interior breakpoints, zero outside the
// open table range), times the phase factor
template <typename L>
__device__ __forceinline__ double law_kT(L &law, double T, double r)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxBp; ++i) {
        if (i >= law.n_hinge) break;
        if (i == 0 ? T > law.b[0] : T >= law.b[i]) s += law.dk[i];
    }
    return s * (r + law.phi * (1.0 - r));
}

template <typename L>
__device__ __forceinline__ double law_c(L &law, double T)
{
    double c = law.c0;
#pragma unroll
    for (int i = 0; i < kMaxBp; ++i) {
        if (i >= law.n_hinge) break;
        c = __builtin_fma(law.dc[i], fmax0(T - law.b[i], 0.0), c);
    }
    if (T >= law.Ts && T <= law.Tl) c += law.lat;
    return c;
}

// 1D Lagrange basis of degree P (1 or 2) on the equispaced nodes of [0,1]
__device__ __forceinline__ double lagrange1(int P, int a, double x)
{
    if (P == 1) return a == 0 ? 1.0 - x : x;
    if (a == 0) return 2.0 * (x - 0.5) * (x - 1.0);
    if (a == 1) return 4.0 * x * (1.0 - x);
    return 2.0 * x * (x - 0.5);
}

}  // namespace
}  // namespace pbf
