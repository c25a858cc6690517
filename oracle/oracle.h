/* Plain CPU oracle of the scan-resolved powder-bed-fusion thermal model.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference that
 * the GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product never does.  It
 * shares no code, header or table with the GPU library.
 *
 * Everything is IEEE double precision, evaluated cell by cell with full
 * (p+1)^3 x (p+1)^3 shape-function tables (no sum factorization, no fusion).
 */
#ifndef PBF_ORACLE_H
#define PBF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    /* uniform box of nx*ny*nz Lagrange Q_degree hexahedra on [0,Lx]x[0,Ly]x[0,Lz] */
    int degree, nx, ny, nz;
    double Lx, Ly, Lz;
    unsigned dirichlet_mask; /* bit f set: face f (x-,x+,y-,y+,z-,z+) is Dirichlet */
    double T_D;
    /* material: piecewise-linear k(T), cp(T) on shared breakpoints */
    int n_bp;
    const double *T_bp, *k_bp, *cp_bp;
    double rho, T_s, T_l, latent, powder_k_factor, powder_depth;
    /* laser: kind -1 off, 0 Gaussian surface flux on z=Lz, 1 cylindrical volume source */
    int laser_kind;
    double radius, absorptivity, h_powder, t_start;
    int n_tracks;
    const double *tracks; /* n_tracks x 8: x0 y0 z0 x1 y1 z1 speed power */
    const double *track_power; /* optional override of the nominal powers (n_tracks) */
    /* radiation and evaporation on the free top surface z = Lz (eqs. bc_radiation,
     * bc_evaporation); off when emissivity == 0 and evap_on == 0 */
    double emissivity, T_inf;
    int evap_on;
    double T_v, C_P, C_T, C_M, h_v, T_h0, dT_max; /* [T] = min(T, T_v + dT_max) */
} or_problem;

/* reference element ------------------------------------------------------- */
int or_gauss_legendre(int n, double *x, double *w);
double or_lagrange(int p, int a, double x);
double or_lagrange_deriv(int p, int a, double x);

/* material law -------------------------------------------------------------- */
double or_liquid_fraction(const or_problem *P, double T);
double or_piecewise_linear(int n, const double *b, const double *v, double T);
double or_conductivity(const or_problem *P, double T, double rc);
double or_capacity(const or_problem *P, double T);

/* laser ----------------------------------------------------------------------- */
int or_beam(const or_problem *P, double t, double *xb, double *yb, double *W, int *track);
double or_volume_source(const or_problem *P, double x, double y, double z, double t);
double or_surface_source(const or_problem *P, double x, double y, double t);
/* layer activation on the whole box P: layers nz_old..nz_new-1 (T to T0, new powder) */
void or_activate_layers(const or_problem *P, int nz_old, int nz_new, double T0, double *T, double *rc);
/* outward heat flux density q_rad + q_evap through the free surface at T */
double or_surface_loss(const or_problem *P, double T);
/* f_RE(T): the surface-loss terms alone, assembled (zero when they are off) */
int or_surface_loss_vector(const or_problem *P, const double *T, double *f);

/* mesh bookkeeping ------------------------------------------------------------ */
int64_t or_n_dofs(const or_problem *P);
int64_t or_n_qp(const or_problem *P);
int or_is_dirichlet(const or_problem *P, int64_t node);
void or_init_history(const or_problem *P, double *rc);

/* explicit scheme -------------------------------------------------------------- */
int or_assemble(const or_problem *P, const double *T, double *rc, double t,
                double *f, double *C, double *fvol);
int or_assemble_lagged(const or_problem *P, const double *T, const double *rc, double t,
                       double *f, double *C, double *fvol);
int or_explicit_steps(const or_problem *P, double *T, double *rc, double t0, double dt, int n);
int or_explicit_step_sampled(const or_problem *P, const double *T, const double *rc, double t,
                             double dt, int n_nodes, const int64_t *nodes, double *T_new);
double or_stability_lambda(const or_problem *P, const double *v0, int iters);

/* implicit scheme ---------------------------------------------------------------- */
int or_capacity_apply(const or_problem *P, const double *Tn, const double *x, double *y);
int or_implicit_step(const or_problem *P, const double *Tn, double *rc, double t, double dt,
                     double cg_rtol, int cg_max_it, double picard_tol, int picard_max_it,
                     double *T_out, int *cg_iters_total, int *picard_iters, double *final_rel_res);
/* Picard matrix: y = (C(T_n)/dt + K(T^i)) x (x zero on Dirichlet nodes, rows zero there) */
int or_picard_apply(const or_problem *P, const double *Tn, const double *Ti, const double *rc, double dt,
                    const double *x, double *y);
/* Newton: y = J(T^i) x (eq. Newton_1, capacity/history/surface losses lagged) */
int or_jacobian_apply(const or_problem *P, const double *Tn, const double *Ti, const double *rc, double dt,
                      const double *x, double *y);
/* R(T) of eq. backward_euler_nonlinear with f_RE lagged at T_n (0 on Dirichlet rows) */
int or_implicit_residual(const or_problem *P, const double *Tn, const double *T, const double *rc, double t,
                         double dt, double *res);
/* backward Euler step by Newton + restarted GMRES(restart), Jacobi on the right */
int or_implicit_step_newton(const or_problem *P, const double *Tn, double *rc, double t, double dt,
                            double lin_rtol, int restart, int lin_max_it, double newton_tol, int newton_max_it,
                            double *T_out, int *lin_iters_total, int *newton_iters, double *final_rel_res);

/* probes and the adjoint -------------------------------------------------------- */
int or_probe(const or_problem *P, const double *T, int n, const double *pts, double *vals);
int or_adjoint_run(const or_problem *P, const double *T0, double t0, double dt, int n_steps,
                   int n_probes, const double *pts, const double *targets,
                   double *J, double *dJ_dW, double *T_final, double *lam0);

#ifdef __cplusplus
}
#endif
/* ---- octree meshes with hanging nodes (octree.c) ---------------------------
 * leaves: n_leaves rows (level, ix, iy, iz), origin in units of the finest cell
 * (coarse cell size / 2^max_level); P->nx.. give the coarse cells.  Dof order:
 * regular nodes sorted by (z, y, x).  History: leaf-major, nq per leaf.
 * hist: 0 update (explicit step), 1 peek, 2 lagged. */
typedef struct or_octree or_octree;
or_octree *or_oct_build(const or_problem *P, int max_level, int64_t n_leaves, const int64_t *leaves);
or_octree *or_oct_build_top(const or_problem *P, int max_level, int64_t n_leaves, const int64_t *leaves,
                            int64_t top);
void or_oct_free(or_octree *O);
int64_t or_oct_n_dofs(const or_octree *O);
int64_t or_oct_n_hanging(const or_octree *O);
int64_t or_oct_n_qp(const or_octree *O);
void or_oct_dof_coords(const or_octree *O, double *xyz);
void or_oct_dirichlet(const or_octree *O, int *flag);
void or_oct_init_history(const or_octree *O, double *rc);
int or_oct_assemble(const or_octree *O, const double *T, double *rc, double t, double *f, double *C,
                    double *fvol, int hist);
int or_oct_explicit_steps(const or_octree *O, double *T, double *rc, double t0, double dt, int n);
double or_oct_stability_lambda(const or_octree *O, const double *v0, int iters);
int or_oct_implicit_step(const or_octree *O, const double *Tn, double *rc, double t, double dt,
                         double cg_rtol, int cg_max_it, double picard_tol, int picard_max_it,
                         double *T_out, int *cg_iters_total, int *picard_iters, double *final_rel_res);
int or_oct_probe(const or_octree *O, const double *T, int n, const double *pts, double *vals);
int or_oct_transfer(const or_octree *Oo, const double *To, const double *rco, const or_octree *On,
                    double *Tn, double *rcn);
int or_oct_transfer_growing(const or_octree *Oo, const double *To, const double *rco, const or_octree *On,
                            double T0, double *Tn, double *rcn);

#endif
