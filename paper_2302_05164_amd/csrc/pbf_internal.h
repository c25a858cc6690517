// Internal definitions shared by the host driver and the HIP kernels of the
// pbftherm library (uniform Lagrange boxes on gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "pbftherm.h"

namespace pbf {

constexpr int kMaxBp = 16;

// ---------------------------------------------------------------------------
// Compile-time 1D tables of the tensor-product element: Gauss points and
// weights on [0,1], Lagrange values on equispaced nodes at the Gauss points,
// and the collocation derivative on the Gauss points (derivative at Gauss point
// q of the Lagrange polynomial through the Gauss points that is one at point
// r).  On a line of a Q_p cell the interpolant is a degree-p polynomial, so its
// derivative at the Gauss points follows exactly from its Gauss-point values.
// ---------------------------------------------------------------------------
constexpr double csqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
    return r;
}

template <int P>
struct Tables {
    static_assert(P == 1 || P == 2, "degree 1 or 2");
    static constexpr int N = P + 1;
    static constexpr double gp(int i)
    {
        // constant tables (the square roots are evaluated at compile time only)
        constexpr double g1[2] = {0.5 - 0.5 / csqrt(3.0), 0.5 + 0.5 / csqrt(3.0)};
        constexpr double g2[3] = {0.5 - csqrt(15.0) / 10.0, 0.5, 0.5 + csqrt(15.0) / 10.0};
        return P == 1 ? g1[i] : g2[i];
    }
    static constexpr double gw(int i)
    {
        if (P == 1) return 0.5;
        return i == 1 ? 8.0 / 18.0 : 5.0 / 18.0;
    }
    // Lagrange polynomial a on the nodes b/P
    static constexpr double lag(int a, double x)
    {
        double v = 1.0;
        for (int b = 0; b <= P; ++b)
            if (b != a) v *= (x - double(b) / P) / (double(a) / P - double(b) / P);
        return v;
    }
    // derivative at x of the Lagrange polynomial through the Gauss points, 1 at point r
    static constexpr double lag_gauss_d(int r, double x)
    {
        double s = 0.0;
        for (int c = 0; c < N; ++c) {
            if (c == r) continue;
            double t = 1.0 / (gp(r) - gp(c));
            for (int b = 0; b < N; ++b)
                if (b != r && b != c) t *= (x - gp(b)) / (gp(r) - gp(b));
            s += t;
        }
        return s;
    }
    // S(q,a) = l_a(x_q): nodes -> Gauss points.  The Q2 midpoint basis function
    // is exactly 1 and the vertex ones exactly 0 at the middle Gauss point.
    static constexpr double S(int q, int a) { return lag(a, gp(q)); }
    static constexpr double D(int q, int r) { return lag_gauss_d(r, gp(q)); }
};

// coefficient "matrices" as types, so that rows can be unrolled at compile time
template <int P> struct TagS  { static constexpr double c(int o, int i) { return Tables<P>::S(o, i); } };
template <int P> struct TagSt { static constexpr double c(int o, int i) { return Tables<P>::S(i, o); } };
template <int P> struct TagD  { static constexpr double c(int o, int i) { return Tables<P>::D(o, i); } };
template <int P> struct TagDt { static constexpr double c(int o, int i) { return Tables<P>::D(i, o); } };

// ---------------------------------------------------------------------------
// material law in hinge form:  v(T) = v0 + sum_i dv_i max(T - b_i, 0), which
// equals the piecewise-linear table with constant extrapolation (the slope
// changes by dv_i at breakpoint b_i).  FP32 variants hold breakpoints and
// thresholds shifted by T_ref.
// ---------------------------------------------------------------------------
template <typename R>
struct Law {
    int n_hinge;
    R b[kMaxBp], dk[kMaxBp], dc[kMaxBp];
    R k0, c0;
    R Ts, Tl, inv_dT, lat;  // lat = latent/(T_l - T_s)
    R phi, rho;
};

// Radiation and evaporation on the free top surface z = Lz (Section 2, eqs.
// bc_radiation and bc_evaporation): outward flux density
//   q(T) = eps sigma_S (T^4 - T_inf^4)
//        + 0.82 C_P exp(-C_T (1/[T] - 1/T_v)) sqrt(C_M/[T]) (h_v + c_p([T]) ([T] - T_h0))
// (second term only where [T] > T_v), [T] = min(T, T_v + dT_max).  on == 0: off.
struct SurfaceLoss {
    int on, evap;
    double eps_sigma, Tinf4;   // eps sigma_S, T_inf^4
    double Tv, inv_Tv, Tmax;   // boiling point, 1/T_v, clamp T_v + dT_max
    double CP82, CT, CM;       // 0.82 C_P, C_T, C_M
    double hv, Th0;            // latent heat of evaporation, enthalpy reference temperature
    const Law<double> *law;    // material law (specific heat of the enthalpy term)
};

// Compact storage of the partial sums at column faces: one entry per face node
// and column parity, in the order in which the face kernels enumerate their
// threads (x-face planes, then y-face planes without x-face nodes, then
// z-segment ends without either), so that those kernels read it coalesced.
// Parity slot s of face node t lives at slots[s * GT + t].
struct FaceMap {
    long long GX, GY, GT;  // x-face nodes, y-face nodes, all face nodes
};

// z-segments of the columns: segment s spans cell layers zb[s] .. zb[s+1]-1
// (zb[0] = 0, zb[MZ] = nz); lengths need not be equal.
constexpr int kMaxSeg = 64;

// Parameters of one cell-kernel launch (passed by value).
template <typename R>
struct CellParams {
    const double *Tin;  // nodal temperatures (state, double)
    double *Tout;       // next state (explicit mode)
    double *fout, *Cout;  // assembled vectors (assemble mode)
    double *hist;       // consolidated fraction of the history layers
    double *slots;      // 8 parity slots of partial sums of f at tile faces
    FaceMap fm;
    int nx, ny, nz, NX, NY, NZ;
    int MX, MY, MZ, ntiles, tiles_per_xcd;  // columns in x, y; z-segments; MX*MY*MZ
    int zb[kMaxSeg + 1];                    // z-segment boundaries (cell layers)
    int hist_cz0, n_hist_cells;
    int hist_write;  // 0: the updated consolidated fraction is used but not stored
    double hx, hy, hz, Lz;
    R detJ, ih2x, ih2y, ih2z;  // h^-2 per direction
    int iso;                   // ih2x == ih2y == ih2z
    double dt, T_D, Tref;
    double ihx, ihy, ihz, dtr;  // 1/h per direction; dt / rho of the nodal law (explicit mode)
    unsigned dmask;
    int laser_on, laser_kind, src_cz0;
    double xb, yb, src_amp, two_over_R2, h_powder;
    const Law<R> *law;          // quadrature-point law (device copy, uniform indices)
    const Law<double> *nlaw;    // nodal capacity law (always double)
    SurfaceLoss re;             // top-surface losses (evaluated in double)
};

// Parameters of the Picard-operator kernels of the implicit step.
struct PicardParams {
    const double *Tc, *Tk, *x1, *x2;  // capacity temperature, conductivity temperature, inputs
    double *yout;
    const double *hist;  // consolidated fraction, lagged (read only)
    double *slots;
    FaceMap fm;
    int nx, ny, nz, NX, NY, NZ;
    int MX, MY, MZ, ntiles, tiles_per_xcd;
    int zb[kMaxSeg + 1];
    int hist_cz0, n_hist_cells;
    double hx, hy, hz, Lz;
    double detJ, ih2x, ih2y, ih2z, inv_dt;
    unsigned dmask;
    int src_on, laser_kind, src_cz0;
    double xb, yb, src_amp, two_over_R2, h_powder;
    const Law<double> *law;
    // per-point coefficient cache of the Krylov applies, [component][point][cell]:
    // 0 capacity weight W rho c(Tc)/dt, 1 conductivity weight W k(Tk, r); Newton
    // also 2 W k_T(Tk, r) and 3..5 the reference gradient of Tk
    double *coef;
    long long ncells;
};

// Parameters of the adjoint cell kernel (reverse of one explicit step).
struct AdjointParams {
    const double *T;     // T_n
    const double *Tn1;   // T_{n+1}
    const double *lam;   // lambda_{n+1}
    double *lam_out;     // lambda_n
    const double *hist;  // r^{n-1} (read only)
    double *mu;          // history adjoint: mu_n in, mu_{n-1} out
    double *slots;
    FaceMap fm;
    double *partials;    // per column tile: source sensitivity of the step
    int nx, ny, nz, NX, NY, NZ;
    int MX, MY, MZ, ntiles, tiles_per_xcd;
    int zb[kMaxSeg + 1];
    int hist_cz0, n_hist_cells;
    double hx, hy, hz, Lz;
    double detJ, ih2x, ih2y, ih2z, dt;
    unsigned dmask;
    int src_on, laser_kind, src_cz0;
    double xb, yb, src_unit, two_over_R2, h_powder;  // src_unit: amplitude per unit W_eff
    const Law<double> *law;
};

// Probe set: containing cell and reference coordinates of each point.
struct ProbeSet {
    const int *cell;      // 3 per probe
    const double *xi;     // 3 per probe
    const double *target; // 1 per probe
    int n, P, NX, NY;
    long long NXY;
};

// Parameters of the tile-face completion kernel.
// Division of 32-bit unsigned numerators n by a fixed divisor d >= 1 with a
// multiply-high: m = floor((2^32 - 1) / d) gives n m / 2^32 > n / d - 1 for
// every n < 2^32, so the estimate is the quotient or one less, and a single
// remainder test corrects it.
struct FastDiv {
    unsigned d, m;
};
inline FastDiv fast_div(unsigned d) { return FastDiv{d, 0xFFFFFFFFu / d}; }

struct HaloParams {
    const double *Tin;
    double *Tout, *fout, *Cout;
    const double *slots;
    const Law<double> *nlaw;
    int P, NX, NY, NZ, SX, SY, MX, MY, MZ;
    int zb[kMaxSeg + 1];  // z-segment boundaries (cell layers)
    long long GX, GY, GZ;  // sizes of the x-, y- and z-face groups
    FastDiv fNX, fNY, fNZ, fSX, fSY;  // divisions of the face-node decode
    double hx, hy, hz, dt, T_D;
    unsigned dmask;
    const unsigned char *dflag;  // per-dof Dirichlet flags (octree meshes), else NULL
};

// tile-face completion of the adjoint kernel
struct AdjointHalo {
    HaloParams h;  // h.Tin = T_n
    const double *Tn1, *lam;
    double *lam_out;
};

// Row sum of the 1D mass matrix at node i of n_nodes (degree P, cell size h):
// the 1D element row sums are (1/2, 1/2) h for Q1 and (1/6, 2/3, 1/6) h for Q2.
__host__ __device__ inline double lumped_mass_1d(int i, int n_nodes, int P, double h)
{
    if (P == 1) return (i == 0 || i == n_nodes - 1) ? 0.5 * h : h;
    if (i & 1) return (2.0 / 3.0) * h;
    return (i == 0 || i == n_nodes - 1) ? (1.0 / 6.0) * h : (1.0 / 3.0) * h;
}

// Cell kernels: a workgroup owns a column of kTX x TY cells (one cell per
// thread) and marches up through a segment of seg_len cell layers.
constexpr int kTX = 16;

// launchers (explicit.hip)
// e0/e1 (optional): events recorded by the dispatch around the kernel's execution
hipError_t launch_cells(int degree, int precision, int mode, int ty, const CellParams<double> &pd,
                        const CellParams<float> &pf, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
// column height in cells (16 x ty columns) and resident workgroups per CU
int column_height();
int resident_columns_per_cu(int ty);
hipError_t launch_halo(int mode, const HaloParams &hp, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
// implicit step (implicit.hip): mode 0 apply, 1 Jacobi diagonal
int picard_column_height();
hipError_t launch_picard(int degree, int mode, const PicardParams &pp, const HaloParams &hp,
                         hipStream_t s);
// per-point coefficients of the Krylov applies (once per Picard/Newton iteration)
hipError_t launch_picard_coef(int degree, bool newton, const PicardParams &pp, hipStream_t s);
// y = C(Tc) x/dt + K(Tk) x (+ L(Tk) x) from the cached coefficients; pp and hp in
// the explicit-kernel geometry (16 x 16 cell columns)
hipError_t launch_picard_capply(int degree, bool newton, const PicardParams &pp, const HaloParams &hp,
                                hipStream_t s);
constexpr int kCoefPicard = 2, kCoefNewton = 6;  // cached components
// vector kernels (vec.hip)
hipError_t launch_fill(double *x, double v, long long n, hipStream_t s);
hipError_t launch_init_dirichlet(double *T, const HaloParams &geom, double T_D, hipStream_t s);
hipError_t launch_init_history(double *rc, int n_hist_cells, int nq1, const int *qz_powder_mask,
                               int hist_layers, int nx, int ny, hipStream_t s);
hipError_t launch_power_dots(const double *f, const double *C, const double *v, double *partials,
                             double *scal, const HaloParams &geom, long long n, hipStream_t s);
hipError_t launch_power_update(const double *f, const double *C, double *v, double *partials,
                               double *scal, const HaloParams &geom, long long n, hipStream_t s);
hipError_t launch_power_scale(double *v, const double *scal, long long n, hipStream_t s);

constexpr int kRedBlocks = 1024;  // blocks of the first reduction stage

// device scalars of the CG iteration (offsets into the scalar array)
enum { CG_RZ0 = 8, CG_RZ1 = 9, CG_RR = 10, CG_PAP = 11, CG_BN2 = 12, CG_DMAX = 13 };
// diagnostics: energy terms (3 values), non-finite count and max |x| (2 values)
enum { SC_ENERGY = 16, SC_FINITE = 20, SC_MG = 24 };
hipError_t launch_energy(const double *Tp, const double *T, const double *f, const double *fv,
                         const double *C, double *partials, double *scal, const HaloParams &geom,
                         long long n, hipStream_t s);
hipError_t launch_finite(const double *x, double *partials, double *scal, long long n, hipStream_t s);
hipError_t launch_cg_start(const double *y, const double *diag, double *r, double *z, double *p,
                           double *x, double *partials, double *scal, const HaloParams &geom,
                           long long n, hipStream_t s);
hipError_t launch_cg_pap(const double *p, const double *Ap, double *partials, double *scal,
                         long long n, hipStream_t s);
hipError_t launch_cg_update(double *x, double *r, double *z, const double *p, const double *Ap,
                            const double *diag, double *partials, double *scal, int rz_old,
                            long long n, hipStream_t s);
hipError_t launch_cg_direction(double *p, const double *z, const double *scal, int rz_old, int rz_new,
                               long long n, hipStream_t s);
hipError_t launch_picard_update(double *Ti, const double *x, double *partials, double *scal,
                                const HaloParams &geom, long long n, hipStream_t s);
hipError_t launch_sub(double *d, const double *a, const double *b, long long n, hipStream_t s);
// geometric multigrid on box lattices (NXf = 2 NXc - 1 per direction)
hipError_t launch_mg_inject(double *c, const double *f, const HaloParams &hc, int NXf, int NYf, hipStream_t s);
hipError_t launch_mg_restrict(double *c, const double *f, const HaloParams &hc, int NXf, int NYf, int NZf,
                              hipStream_t s);
hipError_t launch_mg_prolong_add(double *f, const double *c, const HaloParams &hf, int NXc, int NYc, hipStream_t s);
hipError_t launch_cheb(double *x, double *d, const double *r, const double *diag, double c1, double c2,
                       bool from_zero, long long n, hipStream_t s);
hipError_t launch_axpy(double *y, double a, const double *x, long long n, hipStream_t s);
hipError_t launch_cheb_res(double *x, double *d, const double *b, const double *t, const double *diag, double c1,
                           double c2, long long n, hipStream_t s);
hipError_t launch_mg_restrict_res(double *c, const double *b, const double *t, const HaloParams &hc, int NXf, int NYf,
                                  int NZf, hipStream_t s);
hipError_t launch_seed(double *x, long long n, hipStream_t s);
hipError_t launch_dot_to(const double *a, const double *b, double *partials, double *out, long long n,
                         hipStream_t s);
// history of cells [c0, c1) of a growing box (point-major, stride n_hist_cells):
// 0 (powder) at Gauss levels within depth of the top Lz, else 1
hipError_t launch_layer_history(int degree, double *rc, long long stride, long long c0, long long c1,
                                int cells_per_layer, double hz, double Lz, double depth, hipStream_t s);
// GMRES vector kernels (deterministic reductions); at most kGmMax Krylov vectors
constexpr int kGmMax = 64;
hipError_t launch_mdot(const double *w, const double *V, long long ldv, int k, double *partials, double *out,
                       long long n, hipStream_t s);
hipError_t launch_maxpy(double *w, const double *V, long long ldv, int k, const double *h, long long n,
                        hipStream_t s);
hipError_t launch_gm_update(double *x, const double *V, long long ldv, int k, const double *y, const double *diag,
                            long long n, hipStream_t s);
hipError_t launch_div(double *z, const double *v, const double *d, long long n, hipStream_t s);
hipError_t launch_div_scalar(double *v, const double *w, double h, long long n, hipStream_t s);
hipError_t launch_neg(double *b, const double *y, long long n, hipStream_t s);

// discrete adjoint (adjoint.hip)
int adjoint_column_height();
int adjoint_resident_columns_per_cu();
hipError_t launch_adjoint(int degree, const AdjointParams &ap, const AdjointHalo &hp, hipStream_t s);
// dJdW[track] += sum of the per-tile partials (one workgroup, fixed order)
hipError_t launch_adjoint_finish(const double *partials, int ntiles, double *dJdW, int track,
                                 hipStream_t s);
// dJdP_k = A dJdW_k, dJdA = sum_k P_k dJdW_k
hipError_t launch_adjoint_params(const double *dJdW, const double *powers, double A, int n_tracks,
                                 double *dJdP, double *dJdA, hipStream_t s);
hipError_t launch_probe_values(const ProbeSet &ps, const double *T, double *vals, hipStream_t s);
// J = sum_p (T_h(x_p) - T*_p)^2 into J[0]; lam = dJ/dT (lam zeroed here)
hipError_t launch_objective(const ProbeSet &ps, const double *T, double *J, double *lam, long long n,
                            hipStream_t s);

// ---------------------------------------------------------------------------
// octree meshes with hanging nodes (octree_mesh.cpp on the host, octree.hip)
// ---------------------------------------------------------------------------
// Open-addressing hash map from 64-bit keys (never ~0) to int32 values, for
// the octree's leaf and node lattices (millions of entries).
struct FlatMap {
    static constexpr uint64_t kEmpty = ~0ull;
    std::vector<uint64_t> keys;
    std::vector<int32_t> vals;
    size_t n = 0;
    static uint64_t mix(uint64_t k)
    {
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdULL;
        k ^= k >> 33;
        k *= 0xc4ceb9fe1a85ec53ULL;
        k ^= k >> 33;
        return k;
    }
    void reserve(size_t cap)
    {
        size_t c = 16;
        while (c < 2 * cap) c <<= 1;
        if (c <= keys.size()) return;
        std::vector<uint64_t> ok;
        std::vector<int32_t> ov;
        ok.swap(keys);
        ov.swap(vals);
        keys.assign(c, kEmpty);
        vals.assign(c, -1);
        n = 0;
        for (size_t i = 0; i < ok.size(); ++i)
            if (ok[i] != kEmpty) insert(ok[i], ov[i]);
    }
    // (value stored under k, whether it was inserted now)
    std::pair<int32_t, bool> insert(uint64_t k, int32_t v)
    {
        if (2 * (n + 1) > keys.size()) reserve(keys.size() + 16);
        const size_t mask = keys.size() - 1;
        size_t i = mix(k) & mask;
        while (keys[i] != kEmpty) {
            if (keys[i] == k) return {vals[i], false};
            i = (i + 1) & mask;
        }
        keys[i] = k;
        vals[i] = v;
        ++n;
        return {v, true};
    }
    int32_t find(uint64_t k) const  // -1 if absent
    {
        if (keys.empty()) return -1;
        const size_t mask = keys.size() - 1;
        size_t i = mix(k) & mask;
        while (keys[i] != kEmpty) {
            if (keys[i] == k) return vals[i];
            i = (i + 1) & mask;
        }
        return -1;
    }
};

struct OctMesh {
    int P = 0, maxl = 0, n0[3] = {0, 0, 0};
    double L[3] = {0, 0, 0}, unit[3] = {0, 0, 0};  // unit: finest cell size
    std::vector<int32_t> leaf;                      // (level, ix, iy, iz) per leaf
    int64_t n_cells = 0, n_dofs = 0, n_hanging = 0, n_hist_cells = 0;
    std::vector<int32_t> cidx;                      // NN x n_cells: dof, or -1 - hanging id
    std::vector<int32_t> hstart, hdof;              // expanded constraints (CSR)
    std::vector<double> hw;
    std::vector<int32_t> nstart, nslot;             // per dof: slots a * n_cells + cell
    std::vector<double> nw, mass, coords;
    std::vector<float> nwf;                         // nw in FP32 when every weight is exact there
    bool nw_f32 = false;
    std::vector<int64_t> dof_key;                   // lattice coordinates (step unit / P)
    std::vector<unsigned char> dflag;               // Dirichlet flags
    std::vector<int32_t> cell_hist;                 // history cell of each leaf or -1
    std::vector<double> hist_z;                     // (z origin, z size) per history cell
    FlatMap leaf_map;
    // active top in finest units (the box top, or the current layer of a growing
    // build: leaves cover z < top); growing builds keep history in every leaf
    int64_t top = 0;
    bool growing = false;
};
bool oct_build(OctMesh &m, int P, int maxl, const int n0[3], const double L[3], int64_t n_leaves,
               const int32_t *leaves, std::string &err, int64_t top = -1);
bool oct_layer_leaves(const OctMesh &m, const std::vector<double> &rc_min, int64_t new_top, int64_t d_haz,
                      double r_coarsen, std::vector<int32_t> &out, std::string &err);
void oct_finish(OctMesh &m, unsigned dmask, double powder_depth);
bool oct_path_leaves(const int n0[3], const double L[3], int maxl, double radius, const double *tracks,
                     int n_tracks, double s_lo, double s_hi, std::vector<int32_t> &out, std::string &err);
int32_t oct_locate(const OctMesh &m, const double x_finest[3], double xi[3]);

// device view of an octree mesh
struct OctDev {
    const int32_t *cidx, *hstart, *hdof, *leaf, *cell_hist, *nstart, *nslot;
    const double *hw, *nw, *mass, *hist_z;
    const float *nwf;  // the scatter weights in FP32 (nw_f32), else nw
    const unsigned char *dflag;
    double *E;  // NN x n_cells element vectors
    int n_cells, n_dofs, n_hist_cells, maxl, top_iz, nw_f32;
    double ux, uy, uz, Lz;
};
// parameters of the octree cell passes
struct OctParams {
    OctDev m;
    const double *Tin;        // explicit / assemble
    const double *Tc, *Tk, *x1, *x2;  // Picard apply / diagonal
    double *hist;
    int has_hist, hist_write;
    double inv_dt;
    int laser_on, laser_kind;
    double xb, yb, src_amp, two_over_R2, h_powder;
    const Law<double> *law;
    SurfaceLoss re;  // top-surface losses of leaves with a face on z = Lz
};
// node pass: mode 0 explicit update, 1 assemble f and C~, 2 Picard apply
// (Dirichlet rows 0), 3 Picard diagonal (squared weights, Dirichlet rows 1)
struct OctNodeParams {
    OctDev m;
    const double *Tin;
    double *Tout, *fout, *Cout;
    double dt, T_D;
    const Law<double> *nlaw;
};
hipError_t launch_oct_cells(int degree, const OctParams &p, hipStream_t s);
hipError_t launch_oct_picard(int degree, int mode, const OctParams &p, hipStream_t s);
hipError_t launch_oct_nodes(int mode, const OctNodeParams &p, hipStream_t s);
hipError_t launch_oct_init_history(const OctDev &m, int degree, double powder_depth, double *rc,
                                   hipStream_t s);
// remesh transfer: T_new[i] = old field at (cell[i], xi[3i..]); rc_new[i] =
// src[i] >= 0 ? rc_old[src[i]] : (src[i] == -1 ? 0 : 1)
hipError_t launch_oct_transfer(int degree, const OctDev &old, const double *T_old, const int32_t *cell,
                               const double *xi, int64_t n, double *T_new, double T0, const double *rc_old,
                               const int32_t *src, int64_t n_hist, const int32_t *grp_start, const int32_t *grp_idx,
                               double *rc_new, hipStream_t s);

// binomial checkpoint schedule (revolve.cpp, host only)
bool revolve_schedule(int l, int c, std::vector<pbf_revolve_action> &acts, long long *advances);
long long revolve_min_advances(long long l, int c);

}  // namespace pbf
