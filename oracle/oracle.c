/* Plain CPU oracle of the scan-resolved powder-bed-fusion thermal model.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference that the GPU
 * library is checked against.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load it.  It shares no code with the GPU library.
 *
 * Everything follows the paper's definitions literally, in double precision:
 *  - heat equation, material law and laser source: Section 2 (Mathematical
 *    model), eqs. heat_equation, liquid_fraction, consolidated_fraction,
 *    phase_fractions, material_parameter_interp, heat_soruce_cylindrical and the
 *    boundary conditions init_condition, bc_dirichlet, bc_neumann;
 *  - weak form and Galerkin discretization: Section 3.1, eqs. weak_form,
 *    bubnov_galerkin, semi-discrete;
 *  - explicit forward Euler with the row-sum lumped capacity and its stability
 *    limit: Section 3.2, eqs. forward_euler, forward_euler_taylor,
 *    explicit_time_step;
 *  - implicit backward Euler: Section 3.2, eqs. backward_euler_nonlinear,
 *    Newton_1, Newton_2 (solved here with the symmetric Picard matrix and
 *    Jacobi-preconditioned CG);
 *  - element-level evaluation: Section 4.2, eq. diffusive_term_evaluation and
 *    eq. vector_evaluation, but evaluated with full tables N_a(xi_q) and
 *    grad N_a(xi_q) of size (p+1)^3 x (p+1)^3: no sum factorization.
 * Readings where the paper is silent or garbled:
 *  - the source acts for depths 0 <= z_top - z <= h_powder below the top face
 *    (the printed depth condition cannot hold as written);
 *  - W_eff = absorptivity * nominal power;
 *  - the consolidated fraction is updated before use: r^n = max(r^{n-1}, g(T^n));
 *  - only k depends on the phase; k_m = k_s = k(T), k_p = powder factor * k(T);
 *  - apparent capacity c = c_p(T) + L/(T_l - T_s) on T_s <= T <= T_l;
 *  - lumped capacity C~_i = rho c(T_i) M~_i with M~ the row-sum lumped mass
 *    matrix (M~_ii = sum_j M_ij, M_ij = int N_i N_j): equal to the row sum of
 *    the consistent capacity matrix when c is constant, and positive also for
 *    Q2 elements with a temperature-dependent c (the row sum of the consistent
 *    C(T) is not: Q2 shape functions are negative at some Gauss points);
 *  - the source is evaluated at t_n; track k is active on [t_k, t_{k+1});
 *  - Dirichlet nodes are set to T_D after every step (strong, nodal).
 */
#include "oracle.h"
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* reference element                                                          */
/* ------------------------------------------------------------------------- */

/* Legendre polynomials P_n(z) and P_{n-1}(z) by the three-term recurrence
 * k P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2}. */
static void legendre(int n, double z, double *pn, double *pm)
{
    double a = 1.0, b = z; /* P_0, P_1 */
    for (int k = 2; k <= n; ++k) {
        double c = ((2.0 * k - 1.0) * z * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
    }
    *pn = (n == 0) ? 1.0 : b;
    *pm = (n == 0) ? 0.0 : a;
}

/* Gauss-Legendre rule with n points on [0,1]: roots of P_n found by Newton's
 * method from the Chebyshev guesses, weights 2/((1-z^2) P_n'(z)^2) on [-1,1],
 * then mapped to [0,1] and sorted ascending. */
int or_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 16) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5)), pn, pm, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, &pn, &pm);
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre(n, z, &pn, &pm);
        dp = n * (z * pn - pm) / (z * z - 1.0);
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* 1D Lagrange polynomial l_a of degree p on the equispaced nodes b/p. */
double or_lagrange(int p, int a, double x)
{
    double v = 1.0;
    for (int b = 0; b <= p; ++b)
        if (b != a) v *= (x - (double)b / p) / ((double)a / p - (double)b / p);
    return v;
}

/* Derivative of l_a by the product rule. */
double or_lagrange_deriv(int p, int a, double x)
{
    double s = 0.0;
    for (int c = 0; c <= p; ++c) {
        if (c == a) continue;
        double term = 1.0 / ((double)a / p - (double)c / p);
        for (int b = 0; b <= p; ++b)
            if (b != a && b != c) term *= (x - (double)b / p) / ((double)a / p - (double)b / p);
        s += term;
    }
    return s;
}

/* Shape functions N_a(xi) = l_ax(xi_x) l_ay(xi_y) l_az(xi_z) (eq. bubnov_galerkin
 * with tensor-product Lagrange polynomials), tabulated at the tensor Gauss rule. */
int or_make_ref(int p, ref_elem *R)
{
    if (p < 1 || p > MAXN1 - 1) return -1;
    R->p = p;
    R->n1 = p + 1;
    R->nn = R->n1 * R->n1 * R->n1;
    R->nq = R->nn;
    or_gauss_legendre(R->n1, R->xg, R->wg);
    int n1 = R->n1;
    for (int q = 0; q < R->nq; ++q) {
        int qx = q % n1, qy = (q / n1) % n1, qz = q / (n1 * n1);
        double X = R->xg[qx], Y = R->xg[qy], Z = R->xg[qz];
        R->xi[q][0] = X;
        R->xi[q][1] = Y;
        R->xi[q][2] = Z;
        R->wq[q] = R->wg[qx] * R->wg[qy] * R->wg[qz];
        for (int a = 0; a < R->nn; ++a) {
            int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
            double lx = or_lagrange(p, ax, X), ly = or_lagrange(p, ay, Y), lz = or_lagrange(p, az, Z);
            double dx = or_lagrange_deriv(p, ax, X), dy = or_lagrange_deriv(p, ay, Y),
                   dz = or_lagrange_deriv(p, az, Z);
            R->N[a][q] = lx * ly * lz;
            R->dN[a][q][0] = dx * ly * lz;
            R->dN[a][q][1] = lx * dy * lz;
            R->dN[a][q][2] = lx * ly * dz;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* material law (Section 2)                                                   */
/* ------------------------------------------------------------------------- */

/* eq. liquid_fraction */
double or_liquid_fraction(const or_problem *P, double T)
{
    if (T < P->T_s) return 0.0;
    if (T > P->T_l) return 1.0;
    return (T - P->T_s) / (P->T_l - P->T_s);
}

/* Piecewise-linear interpolation of the table (b_i, v_i): segment i where
 * b_i <= T < b_{i+1}; constant extrapolation outside [b_0, b_{n-1}]. */
double or_piecewise_linear(int n, const double *b, const double *v, double T)
{
    if (n == 1 || T <= b[0]) return v[0];
    if (T >= b[n - 1]) return v[n - 1];
    int i = 0;
    while (i + 1 < n - 1 && T >= b[i + 1]) ++i;
    return v[i] + (T - b[i]) * (v[i + 1] - v[i]) / (b[i + 1] - b[i]);
}

/* slope of the segment picked by or_piecewise_linear (0 outside the table) */
static double pl_slope(int n, const double *b, const double *v, double T)
{
    if (n == 1 || T <= b[0] || T >= b[n - 1]) return 0.0;
    int i = 0;
    while (i + 1 < n - 1 && T >= b[i + 1]) ++i;
    return (v[i + 1] - v[i]) / (b[i + 1] - b[i]);
}

/* eqs. phase_fractions and material_parameter_interp with k_m = k_s = k(T) and
 * k_p = powder factor * k(T). */
double or_conductivity(const or_problem *P, double T, double rc)
{
    double kT = or_piecewise_linear(P->n_bp, P->T_bp, P->k_bp, T);
    double g = or_liquid_fraction(P, T);
    double r_p = 1.0 - rc, r_m = g, r_s = rc - g;
    double k_p = P->powder_k_factor * kT, k_m = kT, k_s = kT;
    return r_p * k_p + r_m * k_m + r_s * k_s;
}

/* apparent heat capacity: c_p(T) plus the latent heat spread over [T_s, T_l] */
double or_capacity(const or_problem *P, double T)
{
    double c = or_piecewise_linear(P->n_bp, P->T_bp, P->cp_bp, T);
    if (T >= P->T_s && T <= P->T_l) c += P->latent / (P->T_l - P->T_s);
    return c;
}

/* d k / d T at fixed rc: the g-terms cancel because k_m = k_s */
static double conductivity_dT(const or_problem *P, double T, double rc)
{
    double s = pl_slope(P->n_bp, P->T_bp, P->k_bp, T);
    double g = or_liquid_fraction(P, T);
    double gp = (T > P->T_s && T < P->T_l) ? 1.0 / (P->T_l - P->T_s) : 0.0;
    double kT = or_piecewise_linear(P->n_bp, P->T_bp, P->k_bp, T);
    /* derivative of (1-rc) f k + g k + (rc-g) k, term by term */
    return (1.0 - rc) * P->powder_k_factor * s + gp * kT + g * s - gp * kT + (rc - g) * s;
}

static double conductivity_drc(const or_problem *P, double T)
{
    double kT = or_piecewise_linear(P->n_bp, P->T_bp, P->k_bp, T);
    /* d/drc of (1-rc) f k + g k + (rc-g) k */
    return -P->powder_k_factor * kT + kT;
}

static double capacity_dT(const or_problem *P, double T)
{
    return pl_slope(P->n_bp, P->T_bp, P->cp_bp, T);
}

static double liquid_fraction_dT(const or_problem *P, double T)
{
    return (T > P->T_s && T < P->T_l) ? 1.0 / (P->T_l - P->T_s) : 0.0;
}

/* ------------------------------------------------------------------------- */
/* laser (eq. heat_soruce_cylindrical)                                        */
/* ------------------------------------------------------------------------- */

static double track_power(const or_problem *P, int k)
{
    return P->track_power ? P->track_power[k] : P->tracks[8 * k + 7];
}

/* Beam centre, effective power and active track at time t.  Tracks are run in
 * order at their own speed; track k is active on [t_k, t_{k+1}). */
int or_beam(const or_problem *P, double t, double *xb, double *yb, double *W, int *track)
{
    if (P->laser_kind < 0 || P->n_tracks <= 0 || t < P->t_start) return 0;
    double tk = P->t_start;
    for (int k = 0; k < P->n_tracks; ++k) {
        const double *tr = P->tracks + 8 * k;
        double dx = tr[3] - tr[0], dy = tr[4] - tr[1], dz = tr[5] - tr[2];
        double len = sqrt(dx * dx + dy * dy + dz * dz);
        double dur = len / tr[6];
        if (t < tk + dur) {
            double s = (t - tk) * tr[6] / len;
            *xb = tr[0] + s * dx;
            *yb = tr[1] + s * dy;
            *W = P->absorptivity * track_power(P, k);
            if (track) *track = k;
            return 1;
        }
        tk += dur;
    }
    return 0;
}

double or_volume_source(const or_problem *P, double x, double y, double z, double t)
{
    double xb, yb, W;
    if (P->laser_kind != 1 || !or_beam(P, t, &xb, &yb, &W, NULL)) return 0.0;
    double depth = P->Lz - z;
    if (depth < 0.0 || depth > P->h_powder) return 0.0;
    double R = P->radius;
    double r2 = (x - xb) * (x - xb) + (y - yb) * (y - yb);
    return 2.0 * W / (OR_PI * R * R * P->h_powder) * exp(-2.0 * r2 / (R * R));
}

double or_surface_source(const or_problem *P, double x, double y, double t)
{
    double xb, yb, W;
    if (P->laser_kind != 0 || !or_beam(P, t, &xb, &yb, &W, NULL)) return 0.0;
    double R = P->radius;
    double r2 = (x - xb) * (x - xb) + (y - yb) * (y - yb);
    return 2.0 * W / (OR_PI * R * R) * exp(-2.0 * r2 / (R * R));
}

/* ------------------------------------------------------------------------- */
/* radiation and evaporation on the free surface (eqs. bc_rad_evap,          */
/* bc_radiation, bc_evaporation)                                              */
/* ------------------------------------------------------------------------- */

int or_surface_loss_on(const or_problem *P) { return P->emissivity != 0.0 || P->evap_on; }

/* q_rad = eps sigma_S (T^4 - T_inf^4); q_evap = mdot(h_v + c([T] - T_h0)) with
 * the evaporation mass flux mdot = 0.82 C_P exp(-C_T (1/[T] - 1/T_v)) sqrt(C_M/[T]),
 * only where [T] > T_v, and [T] = min(T, T_v + dT_max).  c is the specific heat
 * of the law at [T] (no latent part: [T] > T_v lies above the liquidus). */
double or_surface_loss(const or_problem *P, double T)
{
    double q = 0.0;
    if (P->emissivity != 0.0) {
        double T2 = T * T, Ti2 = P->T_inf * P->T_inf;
        q += P->emissivity * OR_SIGMA_SB * (T2 * T2 - Ti2 * Ti2);
    }
    if (P->evap_on) {
        double Tmax = P->T_v + P->dT_max;
        double Tc = T < Tmax ? T : Tmax;
        if (Tc > P->T_v) {
            double mdot = 0.82 * P->C_P * exp(-P->C_T * (1.0 / Tc - 1.0 / P->T_v)) * sqrt(P->C_M / Tc);
            double c = or_piecewise_linear(P->n_bp, P->T_bp, P->cp_bp, Tc);
            q += mdot * (P->h_v + c * (Tc - P->T_h0));
        }
    }
    return q;
}

/* ------------------------------------------------------------------------- */
/* mesh bookkeeping                                                           */
/* ------------------------------------------------------------------------- */

static int64_t NX(const or_problem *P) { return (int64_t)P->degree * P->nx + 1; }
static int64_t NY(const or_problem *P) { return (int64_t)P->degree * P->ny + 1; }
static int64_t NZ(const or_problem *P) { return (int64_t)P->degree * P->nz + 1; }

int64_t or_n_dofs(const or_problem *P) { return NX(P) * NY(P) * NZ(P); }

int64_t or_n_qp(const or_problem *P)
{
    int64_t n1 = P->degree + 1;
    return (int64_t)P->nx * P->ny * P->nz * n1 * n1 * n1;
}

int or_is_dirichlet(const or_problem *P, int64_t node)
{
    int64_t i = node % NX(P), j = (node / NX(P)) % NY(P), k = node / (NX(P) * NY(P));
    unsigned m = P->dirichlet_mask;
    return ((m & 1) && i == 0) || ((m & 2) && i == NX(P) - 1) || ((m & 4) && j == 0) ||
           ((m & 8) && j == NY(P) - 1) || ((m & 16) && k == 0) || ((m & 32) && k == NZ(P) - 1);
}

/* global index of local node a of cell (cx,cy,cz); nodes are numbered
 * lexicographically with x fastest */
static int64_t cell_node(const or_problem *P, int cx, int cy, int cz, int a)
{
    int n1 = P->degree + 1, p = P->degree;
    int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
    return (int64_t)(p * cx + ax) + NX(P) * ((int64_t)(p * cy + ay) + NY(P) * (int64_t)(p * cz + az));
}

/* eq. consolidated_fraction, initial state: 0 (powder) at quadrature points at
 * most powder_depth below the top face, 1 (consolidated) elsewhere. */
void or_init_history(const or_problem *P, double *rc)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    or_make_ref(P->degree, R);
    double hz = P->Lz / P->nz;
    int64_t idx = 0;
    for (int cz = 0; cz < P->nz; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx)
                for (int q = 0; q < R->nq; ++q) {
                    double z = (cz + R->xi[q][2]) * hz;
                    rc[idx++] = (P->Lz - z <= P->powder_depth) ? 0.0 : 1.0;
                }
    free(R);
}

/* Layer activation (Section 4.1) on a box P whose bottom nz_old cell layers are
 * active: layers nz_old .. nz_new-1 become active.  Their new nodes (planes
 * degree*nz_old+1 .. degree*nz_new) start at T0 (Section 2: parts activated
 * later start at the initial temperature); their Gauss points within
 * powder_depth of the new top z = nz_new hz start as powder (r = 0), the others
 * at 1 (eq. consolidated_fraction, initial state).  T and rc cover the whole box
 * (rc cell-major); older cells keep their history. */
void or_activate_layers(const or_problem *P, int nz_old, int nz_new, double T0, double *T, double *rc)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    or_make_ref(P->degree, R);
    double hz = P->Lz / P->nz, Lz_new = nz_new * hz;
    int64_t NXY = NX(P) * NY(P);
    for (int64_t i = NXY * ((int64_t)P->degree * nz_old + 1); i < NXY * ((int64_t)P->degree * nz_new + 1); ++i)
        T[i] = T0;
    for (int cz = nz_old; cz < nz_new; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx) {
                int64_t cell = cx + (int64_t)P->nx * (cy + (int64_t)P->ny * cz);
                for (int q = 0; q < R->nq; ++q) {
                    double z = (cz + R->xi[q][2]) * hz;
                    rc[cell * R->nq + q] = (Lz_new - z <= P->powder_depth) ? 0.0 : 1.0;
                }
            }
    free(R);
}

/* ------------------------------------------------------------------------- */
/* element evaluation (eq. diffusive_term_evaluation, weak_form)              */
/* ------------------------------------------------------------------------- */

/* history handling of cell_eval */
enum { HIST_UPDATE = 0, HIST_PEEK = 1, HIST_LAGGED = 2 };

/* Contributions of one cell to f (diffusion + volume source + surface flux), to
 * the row sums of the unit mass matrix (ce) and to the volume-source part fvol.
 * rc holds the cell's history values.  HIST_UPDATE: r = max(r, g(T_q)) is stored and used (explicit
 * step); HIST_PEEK: the same value is used but not stored; HIST_LAGGED: the
 * stored r is used as it is (implicit step, history lagged at the step start). */
static void cell_eval(const or_problem *P, const ref_elem *R, int cx, int cy, int cz,
                      const double *T, double *rc_cell, int hist, int with_re, double t,
                      double *fe, double *ce, double *fv)
{
    double h[3] = {P->Lx / P->nx, P->Ly / P->ny, P->Lz / P->nz};
    double detJ = h[0] * h[1] * h[2];
    double Te[MAXNN];
    for (int a = 0; a < R->nn; ++a) {
        Te[a] = T[cell_node(P, cx, cy, cz, a)];
        fe[a] = 0.0;
        ce[a] = 0.0;
        fv[a] = 0.0;
    }
    for (int q = 0; q < R->nq; ++q) {
        double Tq = 0.0, gq[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < R->nn; ++a) {
            Tq += R->N[a][q] * Te[a];
            for (int d = 0; d < 3; ++d) gq[d] += R->dN[a][q][d] / h[d] * Te[a];
        }
        double r = rc_cell[q];
        double g = or_liquid_fraction(P, Tq);
        double rn = (hist == HIST_LAGGED) ? r : ((g > r) ? g : r);
        if (hist == HIST_UPDATE) rc_cell[q] = rn;
        double k = or_conductivity(P, Tq, rn);
        double xq = (cx + R->xi[q][0]) * h[0], yq = (cy + R->xi[q][1]) * h[1],
               zq = (cz + R->xi[q][2]) * h[2];
        double src = or_volume_source(P, xq, yq, zq, t);
        double W = R->wq[q] * detJ;
        for (int a = 0; a < R->nn; ++a) {
            double gradN_dot_gradT = 0.0;
            for (int d = 0; d < 3; ++d) gradN_dot_gradT += R->dN[a][q][d] / h[d] * gq[d];
            fe[a] += W * (-k * gradN_dot_gradT + R->N[a][q] * src);
            fv[a] += W * R->N[a][q] * src;
            ce[a] += W * R->N[a][q];
        }
    }
    /* Gaussian surface flux on the top face z = Lz (Neumann input) */
    if (P->laser_kind == 0 && cz == P->nz - 1) {
        int n1 = R->n1;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double xs = (cx + R->xg[i]) * h[0], ys = (cy + R->xg[j]) * h[1];
                double qs = or_surface_source(P, xs, ys, t);
                double W = R->wg[i] * R->wg[j] * h[0] * h[1];
                for (int a = 0; a < R->nn; ++a) {
                    int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
                    double Na = or_lagrange(P->degree, ax, R->xg[i]) *
                                or_lagrange(P->degree, ay, R->xg[j]) *
                                or_lagrange(P->degree, az, 1.0);
                    fe[a] += W * Na * qs;
                    fv[a] += W * Na * qs;
                }
            }
    }
    /* radiation and evaporation: -int N_a q_RE(T) dA over the top face z = Lz */
    if (with_re && or_surface_loss_on(P) && cz == P->nz - 1) {
        int n1 = R->n1;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double Na_s[MAXNN], Ts = 0.0;
                for (int a = 0; a < R->nn; ++a) {
                    int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
                    Na_s[a] = or_lagrange(P->degree, ax, R->xg[i]) * or_lagrange(P->degree, ay, R->xg[j]) *
                              or_lagrange(P->degree, az, 1.0);
                    Ts += Na_s[a] * Te[a];
                }
                double q = or_surface_loss(P, Ts);
                double W = R->wg[i] * R->wg[j] * h[0] * h[1];
                for (int a = 0; a < R->nn; ++a) fe[a] -= W * Na_s[a] * q;
            }
    }
}

/* eq. vector_evaluation: f = sum_e G_e^T f_e; the lumped capacity is
 * C~_i = rho c(T_i) M~_i with M~_i = sum_j M_ij assembled the same way.  rc is
 * updated in place. */
static int assemble_mode(const or_problem *P, const double *T, double *rc, double t, double *f,
                         double *C, double *fvol, int hist);

int or_assemble(const or_problem *P, const double *T, double *rc, double t, double *f, double *C,
                double *fvol)
{
    return assemble_mode(P, T, rc, t, f, C, fvol, HIST_UPDATE);
}

/* f and C~ with the history held fixed and without the surface losses
 * (implicit residual: they enter it lagged at T_n, see or_implicit_step) */
int or_assemble_lagged(const or_problem *P, const double *T, const double *rc, double t, double *f,
                       double *C, double *fvol)
{
    return assemble_mode(P, T, (double *)rc, t, f, C, fvol, HIST_LAGGED);
}

static int assemble_mode(const or_problem *P, const double *T, double *rc, double t, double *f,
                         double *C, double *fvol, int hist)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    int64_t N = or_n_dofs(P);
    memset(f, 0, sizeof(double) * N);
    memset(C, 0, sizeof(double) * N);
    if (fvol) memset(fvol, 0, sizeof(double) * N);
    double fe[MAXNN], ce[MAXNN], fv[MAXNN];
    int64_t cell = 0;
    for (int cz = 0; cz < P->nz; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx, ++cell) {
                cell_eval(P, R, cx, cy, cz, T, rc + cell * R->nq, hist, hist != HIST_LAGGED, t, fe, ce, fv);
                for (int a = 0; a < R->nn; ++a) {
                    int64_t g = cell_node(P, cx, cy, cz, a);
                    f[g] += fe[a];
                    C[g] += ce[a];
                    if (fvol) fvol[g] += fv[a];
                }
            }
    for (int64_t i = 0; i < N; ++i) C[i] *= P->rho * or_capacity(P, T[i]);
    free(R);
    return 0;
}

/* f_RE(T) = -sum over top faces of int N_a q_RE(T) dA (eq. bc_rad_evap), the
 * surface-loss part of f alone */
int or_surface_loss_vector(const or_problem *P, const double *T, double *f)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    int64_t N = or_n_dofs(P);
    memset(f, 0, sizeof(double) * N);
    if (or_surface_loss_on(P)) {
        double h[2] = {P->Lx / P->nx, P->Ly / P->ny};
        int n1 = R->n1, cz = P->nz - 1;
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx)
                for (int j = 0; j < n1; ++j)
                    for (int i = 0; i < n1; ++i) {
                        double Na_s[MAXNN], Ts = 0.0;
                        for (int a = 0; a < R->nn; ++a) {
                            int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
                            Na_s[a] = or_lagrange(P->degree, ax, R->xg[i]) *
                                      or_lagrange(P->degree, ay, R->xg[j]) * or_lagrange(P->degree, az, 1.0);
                            Ts += Na_s[a] * T[cell_node(P, cx, cy, cz, a)];
                        }
                        double q = or_surface_loss(P, Ts);
                        double W = R->wg[i] * R->wg[j] * h[0] * h[1];
                        for (int a = 0; a < R->nn; ++a) f[cell_node(P, cx, cy, cz, a)] -= W * Na_s[a] * q;
                    }
    }
    free(R);
    return 0;
}

/* eq. forward_euler: T_{n+1} = T_n + dt C~^{-1} f(T_n) at free nodes, T_D at
 * Dirichlet nodes; t_n = t0 + n dt. */
int or_explicit_steps(const or_problem *P, double *T, double *rc, double t0, double dt, int n)
{
    int64_t N = or_n_dofs(P);
    double *f = (double *)malloc(sizeof(double) * N), *C = (double *)malloc(sizeof(double) * N);
    if (!f || !C) { free(f); free(C); return -1; }
    for (int s = 0; s < n; ++s) {
        double t = t0 + s * dt;
        or_assemble(P, T, rc, t, f, C, NULL);
        for (int64_t i = 0; i < N; ++i)
            T[i] = or_is_dirichlet(P, i) ? P->T_D : T[i] + dt * f[i] / C[i];
    }
    free(f);
    free(C);
    return 0;
}

/* One explicit step evaluated only at the listed nodes: each node's f and C~ are
 * summed from the cells that contain it.  History is read, not written. */
int or_explicit_step_sampled(const or_problem *P, const double *T, const double *rc, double t,
                             double dt, int n_nodes, const int64_t *nodes, double *T_new)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    double fe[MAXNN], ce[MAXNN], fv[MAXNN], rtmp[MAXNN];
    int p = P->degree, n1 = p + 1;
    for (int s = 0; s < n_nodes; ++s) {
        int64_t g = nodes[s];
        if (or_is_dirichlet(P, g)) { T_new[s] = P->T_D; continue; }
        int64_t i = g % NX(P), j = (g / NX(P)) % NY(P), k = g / (NX(P) * NY(P));
        double fsum = 0.0, csum = 0.0;
        for (int cz = 0; cz < P->nz; ++cz) {
            if (k < (int64_t)p * cz || k > (int64_t)p * cz + p) continue;
            for (int cy = 0; cy < P->ny; ++cy) {
                if (j < (int64_t)p * cy || j > (int64_t)p * cy + p) continue;
                for (int cx = 0; cx < P->nx; ++cx) {
                    if (i < (int64_t)p * cx || i > (int64_t)p * cx + p) continue;
                    int64_t cell = cx + (int64_t)P->nx * (cy + (int64_t)P->ny * cz);
                    memcpy(rtmp, rc + cell * R->nq, sizeof(double) * R->nq);
                    cell_eval(P, R, cx, cy, cz, T, rtmp, HIST_PEEK, 1, t, fe, ce, fv);
                    int a = (int)(i - p * cx) + n1 * ((int)(j - p * cy) + n1 * (int)(k - p * cz));
                    fsum += fe[a];
                    csum += ce[a];
                }
            }
        }
        T_new[s] = T[g] + dt * fsum / (P->rho * or_capacity(P, T[g]) * csum);
    }
    free(R);
    return 0;
}

/* eq. explicit_time_step: largest eigenvalue of C~^{-1} K_diff by power
 * iteration, with the conductivity and capacity fixed at the breakpoint where
 * k/(rho c_p) is largest (the critical parameters), Dirichlet rows removed.
 * The eigenvalue estimate is the Rayleigh quotient v^T K v / v^T C~ v.
 * Returns lambda_max; the critical step is 2/lambda_max. */
double or_stability_lambda(const or_problem *P, const double *v0, int iters)
{
    /* critical parameters */
    int best = 0;
    for (int i = 1; i < P->n_bp; ++i)
        if (P->k_bp[i] / P->cp_bp[i] > P->k_bp[best] / P->cp_bp[best]) best = i;
    double kc = P->k_bp[best], cc = P->cp_bp[best];
    double Tb[1] = {0.0}, kb[1] = {kc}, cb[1] = {cc};
    or_problem L = *P;
    L.n_bp = 1;
    L.T_bp = Tb;
    L.k_bp = kb;
    L.cp_bp = cb;
    L.latent = 0.0;
    L.powder_k_factor = 1.0;
    L.laser_kind = -1;
    L.emissivity = 0.0; /* the criterion involves K_diff only */
    L.evap_on = 0;
    int64_t N = or_n_dofs(P), nq = or_n_qp(P);
    double *v = (double *)malloc(sizeof(double) * N), *f = (double *)malloc(sizeof(double) * N),
           *C = (double *)malloc(sizeof(double) * N), *rc = (double *)malloc(sizeof(double) * nq);
    for (int64_t q = 0; q < nq; ++q) rc[q] = 1.0;
    for (int64_t i = 0; i < N; ++i) v[i] = or_is_dirichlet(P, i) ? 0.0 : v0[i];
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        /* with constant k and no source, f(v) = -K v */
        or_assemble(&L, v, rc, 0.0, f, C, NULL);
        double num = 0.0, den = 0.0, nrm = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            if (or_is_dirichlet(P, i)) continue;
            num += -f[i] * v[i];
            den += C[i] * v[i] * v[i];
        }
        lam = num / den;
        for (int64_t i = 0; i < N; ++i) {
            v[i] = or_is_dirichlet(P, i) ? 0.0 : -f[i] / C[i];
            nrm += v[i] * v[i];
        }
        nrm = sqrt(nrm);
        for (int64_t i = 0; i < N; ++i) v[i] /= nrm;
    }
    free(v);
    free(f);
    free(C);
    free(rc);
    return lam;
}

/* ------------------------------------------------------------------------- */
/* implicit backward Euler (eq. backward_euler_nonlinear)                     */
/* ------------------------------------------------------------------------- */

/* y = C(Tn) x with the consistent capacity matrix C_ab = sum_q W rho c(T_q) N_a N_b */
int or_capacity_apply(const or_problem *P, const double *Tn, const double *x, double *y)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    double h[3] = {P->Lx / P->nx, P->Ly / P->ny, P->Lz / P->nz};
    double detJ = h[0] * h[1] * h[2];
    int64_t N = or_n_dofs(P);
    memset(y, 0, sizeof(double) * N);
    for (int cz = 0; cz < P->nz; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx)
                for (int q = 0; q < R->nq; ++q) {
                    double Tq = 0.0, xq = 0.0;
                    for (int b = 0; b < R->nn; ++b) {
                        int64_t g = cell_node(P, cx, cy, cz, b);
                        Tq += R->N[b][q] * Tn[g];
                        xq += R->N[b][q] * x[g];
                    }
                    double W = R->wq[q] * detJ;
                    double c = or_capacity(P, Tq);
                    for (int a = 0; a < R->nn; ++a)
                        y[cell_node(P, cx, cy, cz, a)] += W * P->rho * c * R->N[a][q] * xq;
                }
    free(R);
    return 0;
}

/* Picard matrix A = C(T_n)/dt + K(T^i): y = A x, and optionally diag(A). The
 * conductivity uses the history rc held at its value from the start of the step.
 * Dirichlet entries of x are ignored (treated as 0) and Dirichlet entries of y
 * are set to 0. */
static void picard_apply(const or_problem *P, const ref_elem *R, const double *Tn, const double *Ti,
                         const double *rc, double dt, const double *x, double *y, double *diag)
{
    double h[3] = {P->Lx / P->nx, P->Ly / P->ny, P->Lz / P->nz};
    double detJ = h[0] * h[1] * h[2];
    int64_t N = or_n_dofs(P);
    if (y) memset(y, 0, sizeof(double) * N);
    if (diag) memset(diag, 0, sizeof(double) * N);
    int64_t cell = 0;
    for (int cz = 0; cz < P->nz; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx, ++cell) {
                int64_t gn[MAXNN];
                double xe[MAXNN];
                for (int a = 0; a < R->nn; ++a) {
                    gn[a] = cell_node(P, cx, cy, cz, a);
                    xe[a] = (x && !or_is_dirichlet(P, gn[a])) ? x[gn[a]] : 0.0;
                }
                for (int q = 0; q < R->nq; ++q) {
                    double Tnq = 0.0, Tiq = 0.0, xq = 0.0, gx[3] = {0, 0, 0};
                    for (int b = 0; b < R->nn; ++b) {
                        Tnq += R->N[b][q] * Tn[gn[b]];
                        Tiq += R->N[b][q] * Ti[gn[b]];
                        xq += R->N[b][q] * xe[b];
                        for (int d = 0; d < 3; ++d) gx[d] += R->dN[b][q][d] / h[d] * xe[b];
                    }
                    double k = or_conductivity(P, Tiq, rc[cell * R->nq + q]);
                    double m = P->rho * or_capacity(P, Tnq) / dt;
                    double W = R->wq[q] * detJ;
                    for (int a = 0; a < R->nn; ++a) {
                        double gg = 0.0, dd = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double da = R->dN[a][q][d] / h[d];
                            gg += da * gx[d];
                            dd += da * da;
                        }
                        if (y) y[gn[a]] += W * (m * R->N[a][q] * xq + k * gg);
                        if (diag) diag[gn[a]] += W * (m * R->N[a][q] * R->N[a][q] + k * dd);
                    }
                }
            }
    for (int64_t i = 0; i < N; ++i)
        if (or_is_dirichlet(P, i)) {
            if (y) y[i] = 0.0;
            if (diag) diag[i] = 1.0;
        }
}

/* Newton Jacobian of the implicit residual (eq. Newton_1 with the capacity,
 * history and surface losses lagged at the step start): y = J x with
 *   J = C(T_n)/dt + K(T^i) + L(T^i),  L_ab = sum_q W k_T(T^i_q, r_q) N_b(q) gradN_a(q) . gradT^i_q,
 * k_T the derivative of k at fixed consolidated fraction (eq. material_parameter_interp).
 * x is taken as zero on Dirichlet nodes, whose rows of y are zero. */
static void newton_apply(const or_problem *P, const ref_elem *R, const double *Tn, const double *Ti,
                         const double *rc, double dt, const double *x, double *y)
{
    double h[3] = {P->Lx / P->nx, P->Ly / P->ny, P->Lz / P->nz};
    double detJ = h[0] * h[1] * h[2];
    int64_t N = or_n_dofs(P);
    picard_apply(P, R, Tn, Ti, rc, dt, x, y, NULL);
    int64_t cell = 0;
    for (int cz = 0; cz < P->nz; ++cz)
        for (int cy = 0; cy < P->ny; ++cy)
            for (int cx = 0; cx < P->nx; ++cx, ++cell) {
                int64_t gn[MAXNN];
                double xe[MAXNN];
                for (int a = 0; a < R->nn; ++a) {
                    gn[a] = cell_node(P, cx, cy, cz, a);
                    xe[a] = !or_is_dirichlet(P, gn[a]) ? x[gn[a]] : 0.0;
                }
                for (int q = 0; q < R->nq; ++q) {
                    double Tiq = 0.0, xq = 0.0, gT[3] = {0, 0, 0};
                    for (int b = 0; b < R->nn; ++b) {
                        Tiq += R->N[b][q] * Ti[gn[b]];
                        xq += R->N[b][q] * xe[b];
                        for (int d = 0; d < 3; ++d) gT[d] += R->dN[b][q][d] / h[d] * Ti[gn[b]];
                    }
                    double kT = conductivity_dT(P, Tiq, rc[cell * R->nq + q]);
                    double W = R->wq[q] * detJ;
                    for (int a = 0; a < R->nn; ++a) {
                        double gg = 0.0;
                        for (int d = 0; d < 3; ++d) gg += R->dN[a][q][d] / h[d] * gT[d];
                        y[gn[a]] += W * kT * xq * gg;
                    }
                }
            }
    for (int64_t i = 0; i < N; ++i)
        if (or_is_dirichlet(P, i)) y[i] = 0.0;
}

int or_picard_apply(const or_problem *P, const double *Tn, const double *Ti, const double *rc, double dt,
                    const double *x, double *y)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    picard_apply(P, R, Tn, Ti, rc, dt, x, y, NULL);
    free(R);
    return 0;
}

int or_jacobian_apply(const or_problem *P, const double *Tn, const double *Ti, const double *rc, double dt,
                      const double *x, double *y)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    newton_apply(P, R, Tn, Ti, rc, dt, x, y);
    free(R);
    return 0;
}

/* Implicit residual R(T) = C(T_n)(T - T_n)/dt - f_diff(T) - f_RE(T_n) - f_vol(t + dt)
 * (eq. backward_euler_nonlinear), zero on Dirichlet rows; fre = f_RE(T_n). */
static void implicit_residual(const or_problem *P, const double *Tn, const double *T, const double *rc,
                              double t1, double dt, const double *fre, double *res, double *work)
{
    int64_t N = or_n_dofs(P);
    double *f = work, *Cl = work + N, *fv = work + 2 * N, *dTn = work + 3 * N, *Cx = work + 4 * N;
    or_assemble_lagged(P, T, rc, t1, f, Cl, fv);
    for (int64_t i = 0; i < N; ++i) dTn[i] = T[i] - Tn[i];
    or_capacity_apply(P, Tn, dTn, Cx);
    for (int64_t i = 0; i < N; ++i) res[i] = or_is_dirichlet(P, i) ? 0.0 : Cx[i] / dt - f[i] - fre[i];
}

int or_implicit_residual(const or_problem *P, const double *Tn, const double *T, const double *rc, double t,
                         double dt, double *res)
{
    int64_t N = or_n_dofs(P);
    double *fre = malloc(sizeof(double) * N), *work = malloc(sizeof(double) * 5 * N);
    or_surface_loss_vector(P, Tn, fre);
    implicit_residual(P, Tn, T, rc, t + dt, dt, fre, res, work);
    free(fre);
    free(work);
    return 0;
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Restarted GMRES(m) for J x = b from x = 0, right-preconditioned with
 * M = diag (Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.5):
 * Arnoldi on J M^{-1} with classical Gram-Schmidt applied twice, Givens
 * rotations on the Hessenberg matrix, stop when the residual estimate
 * |g_{j+1}| <= rtol ||b||; x = M^{-1} V_j y_j at each restart.  Returns the
 * number of Arnoldi steps; *rel gets the final true relative residual. */
static int gmres(const or_problem *P, const ref_elem *R, const double *Tn, const double *Ti, const double *rc,
                 double dt, const double *diag, const double *b, double *x, int m, double rtol, int max_it,
                 double *rel, int *ok)
{
    int64_t N = or_n_dofs(P);
    double *V = malloc(sizeof(double) * N * (m + 1)), *w = malloc(sizeof(double) * N),
           *z = malloc(sizeof(double) * N), *r = malloc(sizeof(double) * N);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double)), *cs = calloc(m, sizeof(double)),
           *sn = calloc(m, sizeof(double)), *g = calloc(m + 1, sizeof(double)), *hc = calloc(m + 1, sizeof(double)),
           *y = calloc(m, sizeof(double));
    double bn = sqrt(dot(N, b, b));
    int it = 0;
    *ok = 0;
    for (int64_t i = 0; i < N; ++i) x[i] = 0.0;
    memcpy(r, b, sizeof(double) * N);
    double rn = bn;
    while (bn > 0 && rn > rtol * bn && it < max_it) {
        for (int64_t i = 0; i < N; ++i) V[i] = r[i] / rn;
        for (int k = 0; k <= m; ++k) g[k] = 0.0;
        g[0] = rn;
        int j;
        for (j = 0; j < m && it < max_it; ++j) {
            for (int64_t i = 0; i < N; ++i) z[i] = V[(int64_t)j * N + i] / diag[i];
            newton_apply(P, R, Tn, Ti, rc, dt, z, w);
            for (int k = 0; k <= j; ++k) hc[k] = 0.0;
            for (int pass = 0; pass < 2; ++pass) { /* classical Gram-Schmidt, twice */
                double hp[64];
                for (int k = 0; k <= j; ++k) hp[k] = dot(N, w, V + (int64_t)k * N);
                for (int k = 0; k <= j; ++k) {
                    for (int64_t i = 0; i < N; ++i) w[i] -= hp[k] * V[(int64_t)k * N + i];
                    hc[k] += hp[k];
                }
            }
            double hn = sqrt(dot(N, w, w));
            ++it;
            for (int64_t i = 0; i < N; ++i) V[(int64_t)(j + 1) * N + i] = hn > 0 ? w[i] / hn : 0.0;
            /* previous rotations, then a new one that zeroes hn */
            for (int k = 0; k < j; ++k) {
                double a = cs[k] * hc[k] + sn[k] * hc[k + 1];
                hc[k + 1] = -sn[k] * hc[k] + cs[k] * hc[k + 1];
                hc[k] = a;
            }
            double den = sqrt(hc[j] * hc[j] + hn * hn);
            cs[j] = den > 0 ? hc[j] / den : 1.0;
            sn[j] = den > 0 ? hn / den : 0.0;
            hc[j] = den;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int k = 0; k <= j; ++k) H[(size_t)k * m + j] = hc[k];
            if (fabs(g[j + 1]) <= rtol * bn || hn == 0.0) { ++j; break; }
        }
        /* y = H^{-1} g (upper triangular j x j), x += M^{-1} V y */
        for (int k = j - 1; k >= 0; --k) {
            double s = g[k];
            for (int l = k + 1; l < j; ++l) s -= H[(size_t)k * m + l] * y[l];
            y[k] = s / H[(size_t)k * m + k];
        }
        for (int64_t i = 0; i < N; ++i) {
            double s = 0.0;
            for (int k = 0; k < j; ++k) s += y[k] * V[(int64_t)k * N + i];
            x[i] += s / diag[i];
        }
        newton_apply(P, R, Tn, Ti, rc, dt, x, w);
        for (int64_t i = 0; i < N; ++i) r[i] = b[i] - w[i];
        rn = sqrt(dot(N, r, r));
    }
    *rel = bn > 0 ? rn / bn : 0.0;
    *ok = !(bn > 0 && rn > rtol * bn);
    free(V); free(w); free(z); free(r); free(H); free(cs); free(sn); free(g); free(hc); free(y);
    return it;
}

/* Backward Euler step by Newton's method (eqs. Newton_1, Newton_2): J(T^i) dT =
 * -R(T^i) solved by restarted GMRES(m) with Jacobi (the diagonal of the Picard
 * matrix C(T_n)/dt + K(T^i)) on the right, to ||r|| <= lin_rtol ||b||; stops
 * when ||dT||_inf <= newton_tol.  The history is committed after convergence.
 * Returns 0, 1 if a linear solve missed its tolerance, 2 if Newton did not converge. */
int or_implicit_step_newton(const or_problem *P, const double *Tn, double *rc, double t, double dt,
                            double lin_rtol, int restart, int lin_max_it, double newton_tol, int newton_max_it,
                            double *T_out, int *lin_iters_total, int *newton_iters, double *final_rel_res)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R) || restart < 1 || restart > 63) { free(R); return -1; }
    int64_t N = or_n_dofs(P);
    double *Ti = T_out;
    double *res = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N), *x = malloc(sizeof(double) * N),
           *diag = malloc(sizeof(double) * N), *fre = malloc(sizeof(double) * N),
           *work = malloc(sizeof(double) * 5 * N), *f = malloc(sizeof(double) * N), *Cl = malloc(sizeof(double) * N);
    or_surface_loss_vector(P, Tn, fre);
    for (int64_t i = 0; i < N; ++i) Ti[i] = or_is_dirichlet(P, i) ? P->T_D : Tn[i];
    int total = 0, status = 0, it;
    double last_rel = 0.0;
    for (it = 0; it < newton_max_it; ++it) {
        implicit_residual(P, Tn, Ti, rc, t + dt, dt, fre, res, work);
        for (int64_t i = 0; i < N; ++i) b[i] = -res[i];
        picard_apply(P, R, Tn, Ti, rc, dt, NULL, NULL, diag);
        int ok = 0;
        total += gmres(P, R, Tn, Ti, rc, dt, diag, b, x, restart, lin_rtol, lin_max_it, &last_rel, &ok);
        if (!ok) status = 1;
        double dmax = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            if (or_is_dirichlet(P, i)) continue;
            Ti[i] += x[i];
            if (fabs(x[i]) > dmax) dmax = fabs(x[i]);
        }
        if (dmax <= newton_tol) { ++it; break; }
    }
    if (it >= newton_max_it && status == 0) status = 2;
    or_assemble(P, Ti, rc, t + dt, f, Cl, NULL); /* commit the history */
    if (lin_iters_total) *lin_iters_total = total;
    if (newton_iters) *newton_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    free(res); free(b); free(x); free(diag); free(fre); free(work); free(f); free(Cl); free(R);
    return status;
}

/* Backward Euler step with Picard iterations A(T^i) dT = -R(T^i), where
 * R(T) = C(T_n)(T - T_n)/dt - f_diff(T) - f_RE(T_n) - f_vol(t + dt), A = C(T_n)/dt + K(T^i)
 * (the surface losses are lagged at T_n, as the paper states for the implicit scheme);
 * the capacity and the consolidated fraction are lagged at the start of the
 * step.  Each linear system is solved by Jacobi-preconditioned CG from zero to
 * ||r|| <= cg_rtol ||b||.  Stops when ||dT||_inf <= picard_tol.  The history is
 * committed after convergence: rc = max(rc, g(T_{n+1})). */
int or_implicit_step(const or_problem *P, const double *Tn, double *rc, double t, double dt,
                     double cg_rtol, int cg_max_it, double picard_tol, int picard_max_it,
                     double *T_out, int *cg_iters_total, int *picard_iters, double *final_rel_res)
{
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    int64_t N = or_n_dofs(P), nq = or_n_qp(P);
    double *Ti = T_out;
    double *res = calloc(N, sizeof(double)), *f = calloc(N, sizeof(double)),
           *Cl = calloc(N, sizeof(double)), *fv = calloc(N, sizeof(double)),
           *Cx = calloc(N, sizeof(double)), *diag = calloc(N, sizeof(double)),
           *x = calloc(N, sizeof(double)), *r = calloc(N, sizeof(double)),
           *z = calloc(N, sizeof(double)), *p = calloc(N, sizeof(double)),
           *Ap = calloc(N, sizeof(double)), *rtmp = malloc(sizeof(double) * nq),
           *dTn = calloc(N, sizeof(double)), *fre = calloc(N, sizeof(double));
    or_surface_loss_vector(P, Tn, fre);
    for (int64_t i = 0; i < N; ++i) Ti[i] = or_is_dirichlet(P, i) ? P->T_D : Tn[i];
    int total = 0, status = 0, it;
    double last_rel = 0.0;
    for (it = 0; it < picard_max_it; ++it) {
        /* residual R(T^i) = C (T^i - T_n)/dt - f_diff(T^i) - f_vol */
        or_assemble_lagged(P, Ti, rc, t + dt, f, Cl, fv); /* f = f_diff + f_vol */
        for (int64_t i = 0; i < N; ++i) dTn[i] = Ti[i] - Tn[i];
        or_capacity_apply(P, Tn, dTn, Cx);
        double bn = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            res[i] = or_is_dirichlet(P, i) ? 0.0 : -(Cx[i] / dt - f[i] - fre[i]);
            bn += res[i] * res[i];
        }
        bn = sqrt(bn);
        /* PCG on A x = res */
        picard_apply(P, R, Tn, Ti, rc, dt, NULL, NULL, diag);
        for (int64_t i = 0; i < N; ++i) {
            x[i] = 0.0;
            r[i] = res[i];
            z[i] = r[i] / diag[i];
            p[i] = z[i];
        }
        double rz = 0.0, rr = 0.0;
        for (int64_t i = 0; i < N; ++i) { rz += r[i] * z[i]; rr += r[i] * r[i]; }
        int k = 0;
        last_rel = bn > 0 ? sqrt(rr) / bn : 0.0;
        while (bn > 0 && sqrt(rr) > cg_rtol * bn && k < cg_max_it) {
            picard_apply(P, R, Tn, Ti, rc, dt, p, Ap, NULL);
            double pAp = 0.0;
            for (int64_t i = 0; i < N; ++i) pAp += p[i] * Ap[i];
            double alpha = rz / pAp;
            rr = 0.0;
            double rz_new = 0.0;
            for (int64_t i = 0; i < N; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * Ap[i];
                z[i] = r[i] / diag[i];
                rz_new += r[i] * z[i];
                rr += r[i] * r[i];
            }
            double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
            ++k;
            last_rel = sqrt(rr) / bn;
        }
        total += k;
        if (bn > 0 && sqrt(rr) > cg_rtol * bn) status = 1; /* CG did not converge */
        double dmax = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            if (or_is_dirichlet(P, i)) continue;
            Ti[i] += x[i];
            if (fabs(x[i]) > dmax) dmax = fabs(x[i]);
        }
        if (dmax <= picard_tol) { ++it; break; }
    }
    if (it >= picard_max_it && status == 0) status = 2;
    /* commit history */
    or_assemble(P, Ti, rc, t + dt, f, Cl, NULL);
    if (cg_iters_total) *cg_iters_total = total;
    if (picard_iters) *picard_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    free(res); free(f); free(Cl); free(fv); free(Cx); free(diag); free(x); free(r); free(z);
    free(p); free(Ap); free(rtmp); free(dTn); free(fre); free(R);
    return status;
}

/* ------------------------------------------------------------------------- */
/* probes and the discrete adjoint                                            */
/* ------------------------------------------------------------------------- */

/* containing cell and reference coordinates of a point; on a shared face the
 * lower cell index is taken */
static void locate(const or_problem *P, const double *pt, int *c, double *xi)
{
    double L[3] = {P->Lx, P->Ly, P->Lz};
    int n[3] = {P->nx, P->ny, P->nz};
    for (int d = 0; d < 3; ++d) {
        double h = L[d] / n[d];
        double s = pt[d] / h;
        int ci = (int)floor(s);
        if (ci > 0 && (double)ci == s) ci -= 1;
        if (ci < 0) ci = 0;
        if (ci > n[d] - 1) ci = n[d] - 1;
        c[d] = ci;
        xi[d] = s - ci;
    }
}

static double shape_at(int p, int a, const double *xi)
{
    int n1 = p + 1;
    int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
    return or_lagrange(p, ax, xi[0]) * or_lagrange(p, ay, xi[1]) * or_lagrange(p, az, xi[2]);
}

/* finite element interpolation T_h(x) = sum_a N_a(xi) T_a (eq. bubnov_galerkin) */
int or_probe(const or_problem *P, const double *T, int n, const double *pts, double *vals)
{
    int nn = (P->degree + 1) * (P->degree + 1) * (P->degree + 1);
    for (int s = 0; s < n; ++s) {
        int c[3];
        double xi[3], v = 0.0;
        locate(P, pts + 3 * s, c, xi);
        for (int a = 0; a < nn; ++a) v += shape_at(P->degree, a, xi) * T[cell_node(P, c[0], c[1], c[2], a)];
        vals[s] = v;
    }
    return 0;
}

/* Discrete adjoint of n_steps explicit steps for J = sum_p (T_h(x_p, t_N) - T*_p)^2,
 * giving dJ/dW_k for the effective power of each track.  Every state is stored
 * (small problems only).  The reverse step differentiates the step map
 *   r^n = max(r^{n-1}, g(T_n)),  T_{n+1} = T_n + dt f(T_n, r^n)/C~(T_n)  (free nodes)
 * with one-sided derivatives: g' = 1/(T_l-T_s) on the open interval, the
 * breakpoint slope of the segment the forward evaluation picked, no derivative of
 * the latent-heat indicator, and the max passing its adjoint to T when
 * g(T_q) > r^{n-1} (to r^{n-1} otherwise, ties included).  The lumped capacity
 * depends on the nodal temperature only: dC~_i/dT_i = rho c'(T_i) M~_i. */
int or_adjoint_run(const or_problem *P, const double *T0, double t0, double dt, int n_steps,
                   int n_probes, const double *pts, const double *targets, double *J,
                   double *dJ_dW, double *T_final, double *lam0)
{
    if (or_surface_loss_on(P)) return -2; /* the adjoint covers the model without surface losses */
    ref_elem *R = (ref_elem *)malloc(sizeof(ref_elem));
    if (!R || or_make_ref(P->degree, R)) { free(R); return -1; }
    int64_t N = or_n_dofs(P), nq = or_n_qp(P);
    double *Ts = (double *)malloc(sizeof(double) * N * (n_steps + 1));
    double *Rs = (double *)malloc(sizeof(double) * nq * (n_steps + 1)); /* r^{n-1} for n = 0..N */
    double *f = (double *)malloc(sizeof(double) * N), *C = (double *)malloc(sizeof(double) * N);
    if (!Ts || !Rs || !f || !C) { free(Ts); free(Rs); free(f); free(C); free(R); return -1; }
    memcpy(Ts, T0, sizeof(double) * N);
    or_init_history(P, Rs);
    for (int n = 0; n < n_steps; ++n) {
        double *Tn = Ts + (int64_t)n * N, *Tn1 = Ts + (int64_t)(n + 1) * N;
        double *rn = Rs + (int64_t)(n + 1) * nq;
        memcpy(rn, Rs + (int64_t)n * nq, sizeof(double) * nq);
        or_assemble(P, Tn, rn, t0 + n * dt, f, C, NULL);
        for (int64_t i = 0; i < N; ++i)
            Tn1[i] = or_is_dirichlet(P, i) ? P->T_D : Tn[i] + dt * f[i] / C[i];
    }
    const double *TN = Ts + (int64_t)n_steps * N;
    if (T_final) memcpy(T_final, TN, sizeof(double) * N);
    /* objective and its gradient with respect to T_N */
    double *lam = (double *)calloc(N, sizeof(double)), *lam_new = (double *)calloc(N, sizeof(double));
    double *mu = (double *)calloc(nq, sizeof(double));
    double *a = (double *)malloc(sizeof(double) * N);
    int nn = R->nn;
    double Jv = 0.0;
    for (int s = 0; s < n_probes; ++s) {
        int c[3];
        double xi[3], v = 0.0;
        locate(P, pts + 3 * s, c, xi);
        for (int q = 0; q < nn; ++q) v += shape_at(P->degree, q, xi) * TN[cell_node(P, c[0], c[1], c[2], q)];
        double e = v - targets[s];
        Jv += e * e;
        for (int q = 0; q < nn; ++q)
            lam[cell_node(P, c[0], c[1], c[2], q)] += 2.0 * e * shape_at(P->degree, q, xi);
    }
    *J = Jv;
    for (int k = 0; k < P->n_tracks; ++k) dJ_dW[k] = 0.0;
    double h[3] = {P->Lx / P->nx, P->Ly / P->ny, P->Lz / P->nz};
    double detJ = h[0] * h[1] * h[2];
    for (int n = n_steps - 1; n >= 0; --n) {
        const double *Tn = Ts + (int64_t)n * N;
        const double *rprev = Rs + (int64_t)n * nq;
        double t = t0 + n * dt;
        /* recompute f and C~ of step n (rc copy: history is not advanced here) */
        double *rtmp = (double *)malloc(sizeof(double) * nq);
        memcpy(rtmp, rprev, sizeof(double) * nq);
        or_assemble(P, Tn, rtmp, t, f, C, NULL);
        free(rtmp);
        for (int64_t i = 0; i < N; ++i) {
            if (or_is_dirichlet(P, i)) {
                a[i] = 0.0;
                lam_new[i] = 0.0;
            } else {
                a[i] = dt * lam[i] / C[i]; /* adjoint of f_i */
                /* identity part, plus the nodal capacity C~_i = rho c(T_i) M~_i:
                 * d(dt f_i / C~_i)/dC~_i * dC~_i/dT_i */
                double dC_dT = C[i] / or_capacity(P, Tn[i]) * capacity_dT(P, Tn[i]);
                lam_new[i] = lam[i] - dt * lam[i] * f[i] / (C[i] * C[i]) * dC_dT;
            }
        }
        double xb, yb, Wb;
        int track = -1;
        int on = or_beam(P, t, &xb, &yb, &Wb, &track);
        int64_t cell = 0;
        for (int cz = 0; cz < P->nz; ++cz)
            for (int cy = 0; cy < P->ny; ++cy)
                for (int cx = 0; cx < P->nx; ++cx, ++cell) {
                    int64_t gn[MAXNN];
                    for (int aa = 0; aa < nn; ++aa) gn[aa] = cell_node(P, cx, cy, cz, aa);
                    for (int q = 0; q < R->nq; ++q) {
                        double Tq = 0.0, gT[3] = {0, 0, 0}, aq = 0.0, ga[3] = {0, 0, 0};
                        for (int bb = 0; bb < nn; ++bb) {
                            double Nb = R->N[bb][q];
                            Tq += Nb * Tn[gn[bb]];
                            aq += Nb * a[gn[bb]];
                            for (int d = 0; d < 3; ++d) {
                                gT[d] += R->dN[bb][q][d] / h[d] * Tn[gn[bb]];
                                ga[d] += R->dN[bb][q][d] / h[d] * a[gn[bb]];
                            }
                        }
                        int64_t qi = cell * R->nq + q;
                        double rp = rprev[qi];
                        double g = or_liquid_fraction(P, Tq);
                        int took_g = g > rp;
                        double rn = took_g ? g : rp;
                        double k = or_conductivity(P, Tq, rn);
                        double W = R->wq[q] * detJ;
                        double ga_gT = ga[0] * gT[0] + ga[1] * gT[1] + ga[2] * gT[2];
                        /* adjoint of k from f_diff = -W k grad N . grad T */
                        double kbar = -W * ga_gT;
                        double Tbar = kbar * conductivity_dT(P, Tq, rn);
                        double rbar = kbar * conductivity_drc(P, Tq) + mu[qi];
                        if (took_g) {
                            Tbar += rbar * liquid_fraction_dT(P, Tq);
                            mu[qi] = 0.0;
                        } else {
                            mu[qi] = rbar;
                        }
                        for (int aa = 0; aa < nn; ++aa) {
                            double gg = 0.0;
                            for (int d = 0; d < 3; ++d) gg += R->dN[aa][q][d] / h[d] * ga[d];
                            lam_new[gn[aa]] += -W * k * gg + Tbar * R->N[aa][q];
                        }
                        /* source is linear in W_eff of the active track */
                        if (on && P->laser_kind == 1) {
                            double xq = (cx + R->xi[q][0]) * h[0], yq = (cy + R->xi[q][1]) * h[1],
                                   zq = (cz + R->xi[q][2]) * h[2];
                            double src = or_volume_source(P, xq, yq, zq, t);
                            dJ_dW[track] += W * aq * src / Wb;
                        }
                    }
                    if (on && P->laser_kind == 0 && cz == P->nz - 1) {
                        int n1 = R->n1;
                        for (int j = 0; j < n1; ++j)
                            for (int i = 0; i < n1; ++i) {
                                double xs = (cx + R->xg[i]) * h[0], ys = (cy + R->xg[j]) * h[1];
                                double qs = or_surface_source(P, xs, ys, t);
                                double Ws = R->wg[i] * R->wg[j] * h[0] * h[1];
                                for (int aa = 0; aa < nn; ++aa) {
                                    int ax = aa % n1, ay = (aa / n1) % n1, az = aa / (n1 * n1);
                                    double Na = or_lagrange(P->degree, ax, R->xg[i]) *
                                                or_lagrange(P->degree, ay, R->xg[j]) *
                                                or_lagrange(P->degree, az, 1.0);
                                    dJ_dW[track] += Ws * Na * qs / Wb * a[gn[aa]];
                                }
                            }
                    }
                }
        double *tmp = lam;
        lam = lam_new;
        lam_new = tmp;
    }
    if (lam0) memcpy(lam0, lam, sizeof(double) * N); /* dJ/dT_0 */
    free(Ts); free(Rs); free(f); free(C); free(lam); free(lam_new); free(mu); free(a);
    free(R);
    return 0;
}
