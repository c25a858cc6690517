/* pbftherm: matrix-free thermal model of laser powder-bed fusion on one AMD
 * Instinct MI355X (gfx950).
 *
 * The library evaluates the nonlinear heat-equation operator of a scan-resolved
 * powder-bed-fusion model with sum factorization on uniform boxes of Lagrange
 * Q1/Q2 hexahedra, and drives it with lumped-mass forward-Euler steps, a
 * backward-Euler step solved by matrix-free Jacobi-preconditioned CG, a
 * stability estimate, probes, and the discrete adjoint of the explicit scheme
 * with binomial checkpointing.  The mathematics is
 * that of Proell et al., "A highly efficient computational approach for
 * part-scale thermal modeling of metal powder bed fusion" (arXiv 2302.05164):
 * the model of Section 2, the discretization and time stepping of Section 3,
 * and the element-level operator evaluation of Section 4.2.
 *
 * Conventions shared by every call:
 *  - Status: every call returns PBF_OK (0) or a negative PBF_E* code and then
 *    leaves a message in pbf_last_error(ctx).  No call aborts the process.
 *  - Memory: the context owns host-side descriptions only (mesh sizes, material,
 *    laser path), copied in by the set-up calls.  All device memory is owned by
 *    the caller: one workspace bound with pbf_bind_device, plus the state arrays
 *    passed to each call.  The library never allocates or frees device memory
 *    and keeps no device pointer across calls except the workspace.
 *  - Streams: device calls take the caller's hipStream_t as `void *stream` and
 *    enqueue their kernels on it.  Calls documented as "synchronizes" wait for
 *    the stream before returning because they return host scalars; every other
 *    device call is asynchronous.
 *  - Layout: nodal vectors (length n_dofs, double) use lexicographic numbering
 *    with x fastest, node (i,j,k) at i + NX*(j + NY*k), NX = degree*nx + 1, ...
 *    The history vector (length n_hist_qp, double) stores the consolidated
 *    fraction of the quadrature points of the top n_hist_layers cell layers (the
 *    only cells that hold powder initially); all other points are consolidated
 *    and carry no storage.  Its order is point-major: index
 *    q*n_hist_cells + c, q = qx + (p+1)*(qy + (p+1)*qz) the tensor Gauss point,
 *    c = cx + nx*(cy + ny*(cz - (nz - n_hist_layers))) the cell.
 *  - Units: SI (m, s, K, W, J).
 *  - Contexts are not thread-safe; distinct contexts are independent.
 */
#ifndef PBFTHERM_H
#define PBFTHERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbf_ctx pbf_ctx;
typedef int pbf_status;

#define PBF_OK 0
#define PBF_EINVAL (-1)     /* invalid argument: null pointer, size, range, order */
#define PBF_ENOMEM (-2)     /* host allocation failed or workspace too small */
#define PBF_EMESH (-3)      /* mesh description not supported */
#define PBF_EDEVICE (-4)    /* HIP runtime error */
#define PBF_ENOCONV (-5)    /* iterative solver did not converge */
#define PBF_ENONFINITE (-6) /* non-finite value detected */
#define PBF_ESTATE (-7)     /* call out of order (e.g. a step before binding) */

#define PBF_PREC_FP64 64    /* operator evaluated in double precision */
#define PBF_PREC_FP32 32    /* operator in single precision on T - T_ref; state,
                               accumulation and update stay double */

/* ---- context ------------------------------------------------------------ */
pbf_status pbf_create(pbf_ctx **out);
void pbf_destroy(pbf_ctx *ctx);
/* Message of the last failing call on ctx (or of pbf_create when ctx is NULL).
 * The pointer stays valid until the next call on ctx. */
const char *pbf_last_error(const pbf_ctx *ctx);

/* ---- mesh and DoF map (Section 3.1, eq. bubnov_galerkin) -------------------
 * Uniform box [0,Lx]x[0,Ly]x[0,Lz] of nx*ny*nz hexahedra with tensor-product
 * Lagrange elements of the given degree (1 or 2) on equispaced nodes and the
 * (degree+1)^3-point Gauss rule.  Resets material, laser and binding. */
pbf_status pbf_mesh_box(pbf_ctx *ctx, int degree, int nx, int ny, int nz, double Lx, double Ly,
                        double Lz);
/* ---- octree meshes with hanging nodes (Section 4.2: the gather includes the
 * hanging-node constraints) -----------------------------------------------------
 * Coarse box of nx*ny*nz cells of [0,Lx]x[0,Ly]x[0,Lz], refined into the given
 * leaves: n_leaves rows (level, ix, iy, iz) of int32, level in [0, max_level]
 * (max_level <= 15), origin in units of the finest cell (coarse cell /
 * 2^max_level), aligned to the leaf size.  The leaves must tile the box without
 * overlap and be 2:1 balanced across faces, edges and vertices (else
 * PBF_EMESH); Morton order is recommended (memory locality).  Nodes of a leaf
 * that lie on a face of a coarser leaf without being one of its nodes hang:
 * their value is the coarse leaf's interpolant there (chains are expanded to
 * regular nodes, the dofs).  Dofs are numbered in order of first appearance;
 * pbf_dof_coords gives their coordinates.  The history is stored for the leaves
 * with a Gauss point at most powder_depth below the top face (point-major over
 * those leaves, in leaf order).  Explicit, assembly, stability, energy and
 * implicit calls work on octrees (FP64); probes and the adjoint need a box.
 * Resets material, laser and binding like pbf_mesh_box. */
pbf_status pbf_mesh_octree(pbf_ctx *ctx, int degree, int nx, int ny, int nz, double Lx, double Ly,
                           double Lz, int max_level, int64_t n_leaves, const int32_t *leaves);
/* ---- growing octree builds (Section 4.1, mesh adaptivity and layer activation)
 * The coarse cells (size h_coarse = 2^max_level h_powder, eq.
 * coarse_fine_relation, so the finest cell is one powder layer thick) span the
 * build chamber [0,Lx]x[0,Ly]x[0,Lz]; the active part is z < top (top in
 * finest cells): cells above it are inactive and carry no dofs, so the leaves
 * tile [0,Lx]x[0,Ly]x[0, top*h_finest] only.  The free surface (source depth,
 * surface losses), the powder depth and the Dirichlet face z+ are at z = top.
 * Every leaf keeps its history (buried unfused powder stays powder).
 * pbf_mesh_octree_growing: like pbf_mesh_octree with the active top `top`.
 * pbf_octree_history_min: rc_min[e] (host, n_leaves) = the smallest
 *   consolidated fraction over the quadrature points of leaf e of the device
 *   history rc (1 for leaves without history).  Synchronizes.
 * pbf_octree_layer_leaves: the leaves after activating the layer
 *   [current top, new_top) (new_top == current top: the current top layer
 *   alone): the current layer and every cell whose distance to it is at most
 *   d_haz finest cells (the paper's d_HAZ = 4 h_powder is 4) are refined to
 *   the finest level; an octet of sibling leaves farther than d_haz below the
 *   current layer is replaced by its parent if the consolidated fraction exceeds
 *   r_coarsen (the paper's 0.9) at every quadrature point of all eight (one
 *   level per activation); the new layer is added at the finest level; then
 *   leaves two or more levels coarser than a leaf they touch (face, edge or
 *   vertex) are split until the tree is 2:1 balanced.  rc_min: per-leaf
 *   minima of the history (host, pbf_octree_history_min; NULL: 1 everywhere);
 *   leaves: host array of 4*capacity int32 in Morton order (NULL: count only).
 *   Host only (no workspace needed).
 * pbf_octree_grow_bytes: prepares the move to such leaves with the active top
 *   new_top (>= the current top), then pbf_octree_remesh binds the new
 *   workspace and transfers: dofs inside the old part take the old field,
 *   dofs above the old top the initial temperature of pbf_init_state; history
 *   points above the old top start as powder (0 within the powder depth of the
 *   new top, 1 below), points of a coarsened parent take the minimum over the
 *   points of its eight old children, the others the nearest Gauss point of
 *   the old leaf containing them.  pbf_octree_remesh_bytes on a growing build
 *   keeps the top and uses the same rules.
 * Errors: PBF_ESTATE without a growing octree or binding, PBF_EMESH for
 * invalid leaf sets, PBF_EINVAL for a top that moves down. */
pbf_status pbf_mesh_octree_growing(pbf_ctx *ctx, int degree, int nx, int ny, int nz, double Lx, double Ly,
                                   double Lz, int max_level, int64_t top, int64_t n_leaves, const int32_t *leaves);
pbf_status pbf_octree_history_min(pbf_ctx *ctx, const double *rc, double *rc_min, void *stream);
pbf_status pbf_octree_layer_leaves(pbf_ctx *ctx, const double *rc_min, int64_t new_top, int64_t d_haz,
                                   double r_coarsen, int32_t *leaves, int64_t capacity, int64_t *n_leaves);
pbf_status pbf_octree_grow_bytes(pbf_ctx *ctx, int64_t new_top, int64_t n_leaves, const int32_t *leaves,
                                 size_t *bytes, int64_t *new_n_dofs, int64_t *new_n_hist_qp);
/* leaves, hanging nodes and finest level of the current octree mesh */
pbf_status pbf_octree_info(const pbf_ctx *ctx, int64_t *n_leaves, int64_t *n_hanging, int *max_level);
/* Remesh onto new leaves (same coarse box, degree and max_level).
 * pbf_octree_remesh_bytes builds the new mesh on the host and returns the size
 * of its workspace and its numbers of dofs and history points (outputs may be
 * NULL except bytes).  pbf_octree_remesh binds that workspace (256-byte aligned)
 * and transfers the state: T_new (new n_dofs) is the old finite element field
 * at the new dofs; each new history point takes the value of the nearest old
 * Gauss point in the old leaf containing it if that point lies within the
 * powder depth, else its initial value.  The old workspace and arrays must stay
 * valid until the call returns; afterwards the context works on the new mesh.
 * Synchronizes. */
pbf_status pbf_octree_remesh_bytes(pbf_ctx *ctx, int64_t n_leaves, const int32_t *leaves, size_t *bytes,
                                   int64_t *new_n_dofs, int64_t *new_n_hist_qp);
pbf_status pbf_octree_remesh(pbf_ctx *ctx, void *workspace, size_t bytes, const double *T_old,
                             const double *rc_old, double *T_new, double *rc_new, void *stream);
/* coordinates of the dofs (host array of 3*n_dofs), boxes and octrees */
pbf_status pbf_dof_coords(const pbf_ctx *ctx, double *xyz);

/* Sizes of the current mesh; any output pointer may be NULL.  n_hist_* depend
 * on the powder depth of the material and are 0 before pbf_set_material.  On a
 * growing box (pbf_set_active_layers) these are the sizes of the whole box,
 * i.e. the lengths of the state arrays T and rc. */
pbf_status pbf_mesh_info(const pbf_ctx *ctx, int64_t *n_dofs, int64_t *n_cells, int64_t *n_qp,
                         int64_t *n_hist_layers, int64_t *n_hist_cells, int64_t *n_hist_qp);

/* ---- growing domain (Section 4.1, layer activation; initial condition of Section 2)
 * A box of nx x ny x nz cells (pbf_mesh_box) of which the bottom nz_active cell
 * layers are active: the domain grows layer by layer, the nodes and cells above
 * the active top carry no DoFs, and the top face of the active cells is the free
 * surface (laser source, surface losses).  Because z is the slowest index the
 * active DoFs are a prefix of the state arrays; every stepping, assembly and
 * diagnostic call works on the active part only.  Call pbf_set_active_layers
 * after pbf_mesh_box and before pbf_bind_device (workspace and state arrays are
 * sized for the whole box; nz_active in [1, nz]).  The consolidated fraction is
 * stored for every cell of the box (point-major, n_hist_cells = nx ny nz), so
 * buried powder keeps its history.  pbf_activate_layers(nz_new) activates the
 * layers nz_active .. nz_new-1: their new nodes start at T0 (the initial
 * condition holds for parts activated later), their Gauss points within the
 * powder depth of the new top start as powder (r = 0), others at 1; older cells
 * keep their history.  Errors: PBF_ESTATE on octrees, after binding
 * (pbf_set_active_layers) or on a box that does not grow (pbf_activate_layers);
 * PBF_EINVAL for nz_new outside (nz_active, nz].  The adjoint entry points
 * refuse a growing box. */
pbf_status pbf_set_active_layers(pbf_ctx *ctx, int nz_active);
pbf_status pbf_active_info(const pbf_ctx *ctx, int *nz_active, int64_t *n_active_dofs, double *Lz_active);
pbf_status pbf_activate_layers(pbf_ctx *ctx, int nz_new, double T0, double *T, double *rc, void *stream);

/* ---- boundary conditions (Section 2, eqs. bc_dirichlet, bc_neumann) ---------
 * Bit f of face_mask makes face f Dirichlet at T_D (bits 0..5: x-, x+, y-, y+,
 * z-, z+); every node on such a face is held at T_D.  Other faces are
 * insulated.  Default: no Dirichlet face. */
pbf_status pbf_set_dirichlet(pbf_ctx *ctx, unsigned face_mask, double T_D);

/* ---- material law (Section 2, eqs. liquid_fraction .. material_parameter_interp)
 * k(T) and c_p(T) are piecewise linear on the shared breakpoints T_bp (strictly
 * increasing, n_bp in [1,16]) and constant outside them.  The liquid fraction is
 * g(T) = clamp((T - T_s)/(T_l - T_s), 0, 1); the consolidated fraction r_c is
 * the running maximum of g (update before use); the conductivity is
 * k = (1 - r_c) k_p + g k_m + (r_c - g) k_s with k_m = k_s = k(T) and
 * k_p = powder_k_factor * k(T).  The heat capacity is the apparent capacity
 * c_p(T) + latent/(T_l - T_s) on T_s <= T <= T_l.  Quadrature points at most
 * powder_depth below the top face start as powder (r_c = 0). */
typedef struct {
    int n_bp;
    const double *T_bp, *k_bp, *cp_bp; /* host arrays of n_bp values, copied */
    double rho, T_s, T_l, latent, powder_k_factor, powder_depth;
} pbf_material;
pbf_status pbf_set_material(pbf_ctx *ctx, const pbf_material *m);

/* ---- laser path (Section 2, eq. heat_soruce_cylindrical) ---------------------
 * Tracks are scanned in order from t_start, each at its own speed; track k is
 * active on [t_k, t_{k+1}); the beam is off outside the path.  W_eff =
 * absorptivity * power.  kind 1 (volume): q = 2 W_eff/(pi R^2 h_powder)
 * exp(-2 r^2/R^2) for depths 0 <= Lz - z <= h_powder, r the distance from the
 * beam axis.  kind 0 (surface): Neumann flux 2 W_eff/(pi R^2) exp(-2 r^2/R^2)
 * on the top face z = Lz.  kind -1: off.  The source of a step from t_n is
 * evaluated at t_n. */
typedef struct {
    double x0[3], x1[3], speed, power;
} pbf_track;
typedef struct {
    int kind;
    double radius, absorptivity, h_powder, t_start;
    int n_tracks;              /* 0..4096 */
    const pbf_track *tracks;   /* host array, copied */
} pbf_laser;
pbf_status pbf_set_laser(pbf_ctx *ctx, const pbf_laser *l);

/* Leaves for pbf_mesh_octree / pbf_octree_remesh refined around a window of a
 * scan path (the octree workload; mesh input, not part of the paper's method):
 * coarse nx x ny x nz cells over [0,Lx]x[0,Ly]x[0,Lz]; every cell within
 * `radius` of the beam path between arc lengths s_lo and s_hi (measured along
 * the tracks in order from the first track's start) reaches max_level.  The
 * path is sampled at points at most half a finest cell apart; a level-l cell is
 * split when its box comes closer than R_{l+1} to a sampled point, with
 * R_max = radius and R_l = R_{l+1} + (diagonal of a level-l cell), which keeps
 * the tree 2:1 balanced across faces, edges and vertices.  leaves: host array
 * of 4*capacity int32 (level, ix, iy, iz rows in Morton order of the origins);
 * *n_leaves receives the count.  With leaves == NULL only the count is
 * returned; a too small capacity returns PBF_ENOMEM.  ctx (may be NULL) takes
 * the error message.  Host only. */
pbf_status pbf_octree_path_leaves(pbf_ctx *ctx, int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                  int max_level, double radius, int n_tracks, const pbf_track *tracks,
                                  double s_lo, double s_hi, int32_t *leaves, int64_t capacity, int64_t *n_leaves);

/* ---- radiation and evaporation (Section 2, eqs. bc_rad_evap, bc_radiation,
 * bc_evaporation) ---------------------------------------------------------------
 * Outward heat flux density through the free top surface z = Lz (boxes) or
 * through the faces of leaves on z = Lz (octrees):
 *   q = emissivity sigma_S (T^4 - T_inf^4)
 *     + 0.82 C_P exp(-C_T (1/[T] - 1/T_v)) sqrt(C_M/[T]) (h_v + c_p([T]) ([T] - T_h0)),
 * the evaporation term only where [T] > T_v, with [T] = min(T, T_v + dT_max) and
 * sigma_S = 5.670374419e-8 W m^-2 K^-4.  c_p is the material's specific heat
 * (pbf_set_material) at [T].  Units: K, Pa (C_P), K s^2 m^-2 (C_M), J/kg (h_v).
 * It enters f (explicit steps, pbf_assemble, pbf_energy's external power) at
 * the current state and the implicit residual lagged at T_n (Section 3.2).  The
 * stability estimate leaves it out (it concerns K_diff only).  s == NULL, or
 * emissivity == 0 with evap_on == 0, switches the term off (the default).
 * Errors: PBF_EINVAL for negative or non-finite constants (with evap_on:
 * T_v, C_M, dT_max must be > 0 and C_P, C_T, h_v >= 0).  The discrete adjoint
 * (pbf_adjoint_step, pbf_gradient_*) does not cover this term and returns
 * PBF_ESTATE while it is on. */
typedef struct {
    double emissivity, T_inf;
    int evap_on;
    double T_v, C_P, C_T, C_M, h_v, T_h0, dT_max;
} pbf_surface_loss;
pbf_status pbf_set_surface_loss(pbf_ctx *ctx, const pbf_surface_loss *s);
/* Replace the nominal track powers (host array of n_tracks) and absorptivity. */
pbf_status pbf_set_track_powers(pbf_ctx *ctx, const double *power, double absorptivity);

/* ---- device binding -------------------------------------------------------------
 * Workspace size for the current mesh; the caller allocates it on the device
 * (256-byte aligned) and binds it together with the stream used for the
 * table uploads (synchronizes).  Binding again replaces the previous one. */
pbf_status pbf_workspace_bytes(const pbf_ctx *ctx, size_t *bytes);
pbf_status pbf_bind_device(pbf_ctx *ctx, void *workspace, size_t bytes, void *stream);

/* T[n_dofs] <- T0 (T_D on Dirichlet nodes); rc[n_hist_qp] <- initial
 * consolidated fraction (0 powder, 1 consolidated).  rc may be NULL when
 * n_hist_qp is 0.  T0 is also the reference temperature of the FP32 operator
 * (it evaluates T - T0).  Needs a mesh and a material; a bound workspace only
 * on octree meshes.  Asynchronous. */
pbf_status pbf_init_state(pbf_ctx *ctx, double T0, double *T, double *rc, void *stream);

/* ---- explicit scheme (Section 3.2, eq. forward_euler) -------------------------
 * n_steps forward-Euler steps T_{n+1} = T_n + dt C~(T_n)^{-1} f(T_n) from time
 * t0 (t_n = t0 + n dt), with C~ the row-sum lumped capacity at T_n and f the
 * diffusion, source and surface-flux terms; Dirichlet nodes are reset to T_D.
 * T (in/out) and T_tmp are device arrays of n_dofs doubles that must not
 * overlap; rc (in/out) is the history.  precision is PBF_PREC_FP64 or
 * PBF_PREC_FP32.  The result is in T.  Asynchronous. */
pbf_status pbf_explicit_steps(pbf_ctx *ctx, double *T, double *T_tmp, double *rc, double t0,
                              double dt, int n_steps, int precision, void *stream);

/* pbf_explicit_steps for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same steps, kernels and results as pbf_explicit_steps, but
 * no workspace has to be bound.  The step's scratch (the device copies of the
 * material law and the column-face partial sums) lives in a static device
 * array of 32 MiB per GPU that the library holds until the process ends; the
 * call allocates nothing.  Box meshes only (PBF_EMESH on octrees).  Meshes
 * whose scratch exceeds 32 MiB are refused with PBF_ENOMEM (Q2 boxes up to
 * about 5M nodes fit); *scratch_bytes (may be NULL) receives the scratch the
 * mesh needs, also when it is refused.  Requires a mesh and a material
 * (PBF_ESTATE otherwise); a bound workspace is neither needed nor touched.
 * Every call on one GPU uses that GPU's array: calls that overlap in time on
 * the same GPU (other streams, other threads, other contexts) race and must
 * be serialized by the caller.  The law is copied into the array at every
 * call, which waits for the stream once before the steps are enqueued; the
 * steps themselves are asynchronous.  The stream must belong to the current
 * device. */
pbf_status pbf_explicit_steps_noalloc(pbf_ctx *ctx, double *T, double *T_tmp, double *rc, double t0, double dt,
                                      int n_steps, int precision, size_t *scratch_bytes, void *stream);

/* f(T) and C~(T) at time t into device arrays f, C (n_dofs doubles each) with the
 * history updated in rc as in a step (eq. vector_evaluation).  Asynchronous. */
pbf_status pbf_assemble(pbf_ctx *ctx, const double *T, double *rc, double t, double *f, double *C,
                        int precision, void *stream);

/* Reference operator for throughput comparisons (Section 5.1 compares the
 * explicit step with a constant-coefficient matrix-free Laplace operator):
 * y = K x with K the stiffness matrix of unit conductivity on the box mesh,
 * K_ij = sum_e integral_e grad N_i . grad N_j (Gauss rule of degree+1 points
 * per direction), evaluated with the same sum-factorized column kernels as
 * the explicit step but with no material law, history, source, capacity or
 * update.  Every node is included (no Dirichlet rows are removed).  x, y:
 * device arrays of n_dofs doubles that must not overlap.  Box meshes only
 * (PBF_EMESH on octrees).  Asynchronous. */
pbf_status pbf_laplace_apply(pbf_ctx *ctx, const double *x, double *y, void *stream);

/* Largest eigenvalue of C~^{-1} K_diff (eq. explicit_time_step) by `iters`
 * power iterations from the device vector v0 (n_dofs), with k and c_p frozen at
 * the breakpoint where k/(rho c_p) is largest; the estimate is the Rayleigh
 * quotient v^T K v / v^T C~ v over free nodes.  dt_crit = 2/lambda.  Uses
 * scratch arrays from the workspace.  Synchronizes. */
pbf_status pbf_stability_lambda(pbf_ctx *ctx, const double *v0, int iters, double *lambda_max,
                                void *stream);

/* Critical explicit time step dt_crit = 2 / lambda_max (eq. explicit_time_step):
 * the forward-Euler scheme is stable for dt < dt_crit.  lambda_max is estimated
 * exactly as in pbf_stability_lambda (same arguments, same power iteration);
 * dt_crit (host) receives 2/lambda_max, and lambda_max (host, may be NULL) the
 * eigenvalue estimate itself.  Returns PBF_ENONFINITE when the estimate is not
 * a positive finite number (for instance a start vector that is zero on every
 * free node).  Synchronizes. */
pbf_status pbf_stability_dt(pbf_ctx *ctx, const double *v0, int iters, double *dt_crit,
                            double *lambda_max, void *stream);

/* Preconditioner of the implicit steps' linear systems (pbf_implicit_step:
 * CG; pbf_implicit_step_newton: GMRES, on the right).  kind 0: Jacobi (the
 * default).  kind 1: one geometric multigrid V-cycle (box meshes): levels Q1 on
 * the same mesh below Q2, then Q1 on meshes coarsened 2x while every cell count
 * is even and more than 4096 nodes remain; each level rediscretizes the Picard
 * matrix C(T_n)/dt + K(T^i) (Section 3.2; for Newton its symmetric part) from
 * the temperatures injected from the finer level, with the consolidated
 * fraction taken as 1; Chebyshev smoothing of D^-1 A of smoothing_degree
 * steps before and after the coarse correction (the same polynomial, so the
 * cycle is symmetric positive definite), eigenvalue bounds from a power
 * iteration at the first iteration of each step, restriction = transposed
 * trilinear interpolation, coarsest level by a Chebyshev polynomial of
 * coarse_degree steps.  Only the iteration changes, not the solution (each
 * linear solve still stops at the relative residual asked for).  Call after
 * the mesh, Dirichlet faces and material and before pbf_bind_device (the
 * coarse levels take their memory from the workspace, which grows).  Errors:
 * PBF_ESTATE before mesh and material, PBF_EMESH on octrees and growing boxes,
 * PBF_EINVAL for degrees outside [1, 8] (smoothing) and [1, 64] (coarse). */
pbf_status pbf_set_implicit_preconditioner(pbf_ctx *ctx, int kind, int smoothing_degree, int coarse_degree);
/* Forcing terms of pbf_implicit_step_newton's linear solves.  kind 0 (the
 * default): every Newton system is solved to the relative residual lin_rtol.
 * kind 1: inexact Newton with the Eisenstat-Walker forcing term (choice 2):
 * eta_0 = 0.1, eta_k = 0.9 (|R(T^k)| / |R(T^k-1)|)^2, safeguarded by 0.9
 * eta_{k-1}^2 when that exceeds 0.1, at most 0.1 and at least lin_rtol; early
 * systems are solved loosely, the last ones to lin_rtol.  The Newton stopping
 * rule (max |dT| <= newton_tol) is unchanged. */
pbf_status pbf_set_newton_forcing(pbf_ctx *ctx, int kind);

/* ---- implicit scheme (Section 3.2, eqs. backward_euler_nonlinear, Newton_1, Newton_2)
 * One backward-Euler step from T_n (time t) to T_out (time t + dt), solving
 *   R(T) = C(T_n)(T - T_n)/dt - f_diff(T) - f_vol(t + dt) = 0
 * at free nodes (Dirichlet nodes held at T_D) by Picard iterations
 * (C(T_n)/dt + K(T^i)) dT = -R(T^i): the symmetric part of the Jacobian of
 * eq. Newton_1, applied matrix-free (Section 4.2, eq. matrix_free_eval without
 * the L_e term).  C is the consistent apparent-capacity matrix at T_n; the
 * consolidated fraction is held at its value in rc during the step and then
 * committed as max(rc, g(T_out)).  Each linear system is solved from zero by
 * Jacobi-preconditioned CG to ||r|| <= cg_rtol ||b|| (at most cg_max_it
 * iterations); Picard stops when max|dT| <= picard_tol (at most picard_max_it).
 * T_n and T_out: device arrays of n_dofs doubles (distinct); rc in/out.
 * Outputs: total CG iterations, Picard iterations, relative residual of the last
 * CG solve.  Returns PBF_ENOCONV (with T_out holding the last iterate) when a
 * limit is reached.  Synchronizes (one scalar read per CG iteration). */
pbf_status pbf_implicit_step(pbf_ctx *ctx, const double *T_n, double *T_out, double *rc, double t,
                             double dt, double cg_rtol, int cg_max_it, double picard_tol,
                             int picard_max_it, int *cg_iters_total, int *picard_iters,
                             double *final_rel_res, void *stream);

/* ---- implicit step by Newton's method (Section 3.2, eqs. Newton_1, Newton_2) ---
 * The same step and residual as pbf_implicit_step, solved with the full Jacobian
 *   J(T^i) = C(T_n)/dt + K(T^i) + L(T^i),
 *   L_ab = sum_q W_q k_T(T^i_q, r_q) N_b(x_q) grad N_a(x_q) . grad T^i(x_q)
 * (the nonsymmetric term of eq. matrix_free_eval; k_T is dk/dT at fixed
 * consolidated fraction, the slope of the table segment containing T:
 * right-continuous at interior breakpoints, zero outside the open table range).
 * Each Newton system J dT = -R(T^i) is solved from zero by restarted GMRES(restart)
 * (Arnoldi with classical Gram-Schmidt applied twice, Givens rotations) with
 * Jacobi on the right, M = diag(C(T_n)/dt + K(T^i)), to ||r|| <= lin_rtol ||b||
 * (at most lin_max_it Arnoldi steps); Newton stops when max|dT| <= newton_tol
 * (at most newton_max_it iterations).  Boxes only (PBF_ESTATE on octrees).
 * work: caller-owned device buffer, 256-byte aligned, of pbf_newton_work_bytes
 * (restart + 1 Krylov vectors of n_dofs doubles plus reduction scratch);
 * restart in [1, 63].  Outputs and errors as pbf_implicit_step (PBF_ENOCONV when
 * a limit is reached, T_out holding the last iterate).  Synchronizes (a few
 * scalar reads per Arnoldi step). */
pbf_status pbf_newton_work_bytes(pbf_ctx *ctx, int restart, size_t *bytes);
pbf_status pbf_implicit_step_newton(pbf_ctx *ctx, const double *T_n, double *T_out, double *rc, double t,
                                    double dt, double lin_rtol, int restart, int lin_max_it, double newton_tol,
                                    int newton_max_it, void *work, size_t work_bytes, int *lin_iters_total,
                                    int *newton_iters, double *final_rel_res, void *stream);

/* ---- probes and objective (Section 3.1, eq. bubnov_galerkin) -----------------
 * pbf_set_probes: n points (host array pts[3n], inside the box) and targets
 * (host array of n, may be NULL for zeros), n in [0, 4096], copied and uploaded
 * into the workspace; needs a bound device.  A point on a face shared by two
 * cells is taken in the cell of lower index.  Synchronizes.
 * pbf_probe: vals[p] = T_h(x_p) = sum_a N_a(x_p) T_a, device array of n.
 * pbf_objective: J[0] = sum_p (T_h(x_p) - target_p)^2 (device scalar) and
 * lam = dJ/dT (device array of n_dofs, overwritten).  Asynchronous. */
pbf_status pbf_set_probes(pbf_ctx *ctx, int n, const double *pts, const double *targets, void *stream);
pbf_status pbf_probe(pbf_ctx *ctx, const double *T, double *vals, void *stream);
pbf_status pbf_objective(pbf_ctx *ctx, const double *T, double *J, double *lam, void *stream);

/* ---- diagnostics -----------------------------------------------------------------
 * pbf_energy: energy terms of the explicit step from T_prev (time t, step dt) to
 * T, with rc the history after that step (read only).  With f = f_diff + f_vol
 * and C~ evaluated at T_prev as in the step (Section 3.2, eq. forward_euler),
 * over the free nodes:
 *   out[0] = sum C~_i (T_i - T_prev,i)   change of stored heat,
 *   out[1] = sum f_vol,i                 absorbed laser power,
 *   out[2] = -sum f_diff,i               heat flow into the Dirichlet nodes,
 *   out[3] = out[0] - dt (out[1] - out[2])  (zero up to round-off for a step
 *            of pbf_explicit_steps).
 * Since the diffusion rows sum to zero, out[2] equals the sum of f_diff over the
 * Dirichlet nodes.  Host array out[4].  Uses workspace scratch.  Synchronizes.
 * pbf_check_finite: *ok = 1 if all n values of the device array x are finite,
 * *maxabs = max |x_i| over the finite ones; returns PBF_ENONFINITE otherwise.
 * Synchronizes. */
pbf_status pbf_energy(pbf_ctx *ctx, const double *T_prev, const double *T, const double *rc, double t,
                      double dt, double out[4], void *stream);
pbf_status pbf_check_finite(pbf_ctx *ctx, const double *x, int64_t n, int *ok, double *maxabs,
                            void *stream);

/* ---- discrete adjoint of the explicit scheme -------------------------------------
 * Reverse of one step of eq. forward_euler (Section 3.2) with the law of
 * Section 2: the step maps (T_n, r^{n-1}) to r^n = max(r^{n-1}, g(T_n)) and
 * T_{n+1} = T_n + dt f(T_n, r^n)/C~(T_n).  Given lambda_{n+1} = dJ/dT_{n+1} and
 * mu_n = dJ/dr^n from later steps, pbf_adjoint_step writes lambda_n = dJ/dT_n
 * into lam (n_dofs, must not overlap lam_next), replaces mu (n_hist_qp) by
 * mu_{n-1}, and adds the sensitivity of J to the effective power W_eff of the
 * track active at t_n to dJdW[track] (device array of n_tracks).  T_n and
 * rc_prev = r^{n-1} are the step's input state, T_next = T_{n+1} its output
 * (all read only; the capacity term uses dt f/C~ = T_{n+1} - T_n).  Derivative
 * conventions at non-smooth points: the slope of the table segment that the
 * forward evaluation used (zero outside the table), g' = 1/(T_l - T_s) on the
 * open melting interval, no derivative of the latent-heat box, and the max
 * passes the adjoint to T where g(T) > r^{n-1} (to r^{n-1} otherwise, ties
 * included).  FP64.  Asynchronous. */
pbf_status pbf_adjoint_step(pbf_ctx *ctx, const double *T_n, const double *T_next, const double *rc_prev,
                            const double *lam_next, double *lam, double *mu, double t_n, double dt,
                            double *dJdW, void *stream);

/* ---- binomial checkpointing (reverse of n_steps explicit steps) ----------------
 * Schedule of a reversal with n_snaps state slots (slot 0 holds the initial
 * state): the repetition number r is the smallest with C(n_snaps + r, r) >=
 * n_steps and the number of forward steps is r n_steps - C(n_snaps + r, r - 1),
 * the minimum for that memory (Griewank's binomial checkpointing).  Actions:
 *   ADVANCE(step):  forward steps from the current state up to `step`;
 *   STORE(step, slot): copy the current state (step) into `slot`;
 *   RESTORE(step, slot): make the state in `slot` (step) current;
 *   TURN(step):     adjoint step at the current state `step`.
 * TURN steps come in the order n_steps-1, ..., 0.  Host only: pbf_revolve_schedule
 * counts (actions may be NULL) or lists at most max_actions actions. */
#define PBF_ACT_ADVANCE 1
#define PBF_ACT_STORE 2
#define PBF_ACT_RESTORE 3
#define PBF_ACT_TURN 4
typedef struct {
    int kind, step, slot;
} pbf_revolve_action;
pbf_status pbf_revolve_schedule(int n_steps, int n_snaps, pbf_revolve_action *actions,
                                int max_actions, int *n_actions, int64_t *n_advances);

/* Gradient of J(T_N) (pbf_objective with the current probes) after n_steps
 * explicit FP64 steps from (T0, rc0) at time t0, with respect to the track
 * powers and the absorptivity, by the adjoint steps above under the binomial
 * schedule with n_snaps slots held in the caller's device buffer `work`
 * (pbf_adjoint_work_bytes; 256-byte aligned).
 * pbf_gradient_forward: runs the forward sweep (taking the snapshots), the
 * last step and the objective: T_N (n_dofs, may be NULL) and J (device scalar,
 * may be NULL).  T0/rc0 are read only.
 * pbf_gradient_backward: with the same work buffer and arguments, runs the
 * reversal: dJdW[k] (device, n_tracks) = dJ/dW_eff,k, dJdP[k] = A dJdW[k]
 * (track powers P), dJdA[0] = sum_k P_k dJdW[k] (absorptivity A),
 * lam0 = dJ/dT0 (n_dofs); any output may be NULL.  n_advances (host, may be
 * NULL) receives the forward steps of both sweeps.  Asynchronous, except that
 * the forward sweep synchronizes once to upload the powers. */
pbf_status pbf_adjoint_work_bytes(const pbf_ctx *ctx, int n_snaps, size_t *bytes);
pbf_status pbf_gradient_forward(pbf_ctx *ctx, const double *T0, const double *rc0, double t0,
                                double dt, int n_steps, int n_snaps, void *work, size_t work_bytes,
                                double *T_N, double *J, void *stream);
pbf_status pbf_gradient_backward(pbf_ctx *ctx, double t0, double dt, int n_steps, int n_snaps,
                                 void *work, size_t work_bytes, double *dJdW, double *dJdP,
                                 double *dJdA, double *lam0, int64_t *n_advances, void *stream);

/* ---- kernel timing (instrumentation) ------------------------------------------
 * pbf_timing_begin: from now on pbf_explicit_steps (and pbf_laplace_apply)
 * has the dispatches of the cell kernel and of the tile-face kernel record HIP
 * start/stop events on the caller's stream (execution time of each kernel) on
 * every `every`-th step or apply (1: all), for at most max_steps timed ones
 * (host-side event pool, created here).
 * pbf_timing_end: waits for the recorded events and returns the average
 * duration in milliseconds of the cell kernel and of the tile-face kernel and
 * the number of timed steps; releases the events.  Synchronizes. */
pbf_status pbf_timing_begin(pbf_ctx *ctx, int max_steps, int every);
pbf_status pbf_timing_end(pbf_ctx *ctx, double *cell_ms, double *face_ms, int64_t *n_steps);

#ifdef __cplusplus
}
#endif
#endif
