/* Oracle on octree meshes with hanging nodes.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): slow, obviously correct, shares no
 * code with the GPU library.
 *
 * The paper's meshes are adaptively refined hexahedral octrees whose fine cells
 * meet coarse neighbours with hanging nodes (Section 4.2: the gather G_e then
 * includes the constraint interpolation; hanging nodes make the evaluation
 * more expensive).  Continuity is imposed as follows:
 *  - the mesh is a list of leaves (level l, origin in units of the finest
 *    cell); a leaf of level l has size h0 / 2^l in each direction;
 *  - its nodes are the (p+1)^3 equispaced Lagrange nodes; a node of some leaf
 *    that lies on the closed box of another leaf L without being one of L's
 *    nodes is hanging: its value is the interpolant of L at that point,
 *    sum_a N_a^L(x) T_a^L (only L's face/edge nodes have non-zero weights);
 *  - constraints whose masters are themselves hanging are expanded until only
 *    regular nodes (the degrees of freedom) remain;
 *  - the element vector of a leaf is scattered with the transposed
 *    constraints: f_i += w_ai fe_a, and the lumped mass M~_i = sum_e sum_a w_ai
 *    int N_a (row sums of P^T M P, since the constraints reproduce constants).
 * Everything else (material law, source, lumped capacity C~_i = rho c(T_i) M~_i,
 * history per quadrature point, Dirichlet nodes on the masked faces) is as on
 * boxes.  Hanging-node detection is a brute-force search over all leaves. */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#include "oracle_internal.h"

struct or_octree {
    or_problem P;
    int maxl, p;
    ref_elem R;
    int64_t nl;
    int64_t *leaf;      /* (level, ix, iy, iz) per leaf */
    double unit[3];     /* finest cell size */
    int64_t nnodes;
    int64_t *key;       /* lattice coordinates of nodes (lattice step unit/p), sorted z, y, x */
    int64_t *cnode;     /* nl * nn node ids */
    int64_t *dof;       /* node -> dof or -1 */
    int64_t ndofs;
    int64_t *dnode;     /* dof -> node */
    int64_t *cs;        /* closure of node k: entries cs[k] .. cs[k+1]-1 */
    int64_t *cd;
    double *cw;
    double *mass;       /* lumped mass per dof */
    int64_t top;        /* active top in finest units (the box top unless the part grows) */
};

static int64_t leaf_span(const or_octree *O, int64_t e) /* leaf size in lattice steps */
{
    return (int64_t)O->p << (O->maxl - O->leaf[4 * e]);
}

static int cmp_key(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    for (int d = 2; d >= 0; --d)
        if (x[d] != y[d]) return x[d] < y[d] ? -1 : 1;
    return 0;
}

static int64_t find_node(const or_octree *O, const int64_t *k)
{
    int64_t lo = 0, hi = O->nnodes - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = cmp_key(O->key + 3 * mid, k);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static void leaf_geometry(const or_octree *O, int64_t e, double *x0, double *h)
{
    int64_t s = (int64_t)1 << (O->maxl - O->leaf[4 * e]);
    for (int d = 0; d < 3; ++d) {
        x0[d] = O->leaf[4 * e + 1 + d] * O->unit[d];
        h[d] = s * O->unit[d];
    }
}

/* closure of node k as (dof, weight) lists; hang[k] = leaf that constrains k or -1 */
static int expand(or_octree *O, const int64_t *hang, int64_t k, int64_t **ld, double **lw, int64_t *ln)
{
    if (ln[k] >= 0) return 0;
    if (hang[k] < 0) {
        ld[k] = malloc(sizeof(int64_t));
        lw[k] = malloc(sizeof(double));
        ld[k][0] = O->dof[k];
        lw[k][0] = 1.0;
        ln[k] = 1;
        return 0;
    }
    int64_t e = hang[k], span = leaf_span(O, e);
    double xi[3];
    for (int d = 0; d < 3; ++d) xi[d] = (double)(O->key[3 * k + d] - O->leaf[4 * e + 1 + d] * O->p) / span;
    int64_t cap = 16, n = 0;
    int64_t *od = malloc(sizeof(int64_t) * cap);
    double *ow = malloc(sizeof(double) * cap);
    int n1 = O->p + 1;
    for (int a = 0; a < O->R.nn; ++a) {
        int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
        double w = or_lagrange(O->p, ax, xi[0]) * or_lagrange(O->p, ay, xi[1]) * or_lagrange(O->p, az, xi[2]);
        if (w == 0.0) continue;
        int64_t m = O->cnode[e * O->R.nn + a];
        if (expand(O, hang, m, ld, lw, ln)) return -1;
        for (int64_t j = 0; j < ln[m]; ++j) {
            int64_t t;
            for (t = 0; t < n; ++t)
                if (od[t] == ld[m][j]) break;
            if (t == n) {
                if (n == cap) {
                    cap *= 2;
                    od = realloc(od, sizeof(int64_t) * cap);
                    ow = realloc(ow, sizeof(double) * cap);
                }
                od[n] = ld[m][j];
                ow[n] = 0.0;
                ++n;
            }
            ow[t] += w * lw[m][j];
        }
    }
    ld[k] = od;
    lw[k] = ow;
    ln[k] = n;
    return 0;
}

void or_oct_free(or_octree *O)
{
    if (!O) return;
    free(O->leaf); free(O->key); free(O->cnode); free(O->dof); free(O->dnode);
    free(O->cs); free(O->cd); free(O->cw); free(O->mass);
    free(O);
}

or_octree *or_oct_build(const or_problem *P, int max_level, int64_t n_leaves, const int64_t *leaves)
{
    return or_oct_build_top(P, max_level, n_leaves, leaves, (int64_t)P->nz << max_level);
}

/* An octree whose leaves cover the box only up to z = top (finest units): the
 * active part of a growing build (Section 4.1: cells above the current layer
 * carry no dofs).  The free surface, the source depth and the powder depth are
 * measured from z = top, and Dirichlet nodes of face z+ lie on z = top. */
or_octree *or_oct_build_top(const or_problem *P, int max_level, int64_t n_leaves, const int64_t *leaves,
                            int64_t top)
{
    or_octree *O = calloc(1, sizeof(or_octree));
    if (!O || or_make_ref(P->degree, &O->R)) { free(O); return NULL; }
    O->P = *P;
    O->maxl = max_level;
    O->p = P->degree;
    O->nl = n_leaves;
    O->leaf = malloc(sizeof(int64_t) * 4 * n_leaves);
    memcpy(O->leaf, leaves, sizeof(int64_t) * 4 * n_leaves);
    O->unit[0] = P->Lx / P->nx / (double)((int64_t)1 << max_level);
    O->unit[1] = P->Ly / P->ny / (double)((int64_t)1 << max_level);
    O->unit[2] = P->Lz / P->nz / (double)((int64_t)1 << max_level);
    O->top = top;
    O->P.Lz = (double)top * O->unit[2];  /* the active top */
    int nn = O->R.nn, n1 = O->p + 1;
    /* nodes: all leaf nodes, sorted and unique */
    int64_t *all = malloc(sizeof(int64_t) * 3 * n_leaves * nn);
    for (int64_t e = 0; e < n_leaves; ++e) {
        int64_t step = (int64_t)1 << (max_level - leaves[4 * e]);
        for (int a = 0; a < nn; ++a) {
            int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
            int64_t *k = all + 3 * (e * nn + a);
            k[0] = leaves[4 * e + 1] * O->p + ax * step;
            k[1] = leaves[4 * e + 2] * O->p + ay * step;
            k[2] = leaves[4 * e + 3] * O->p + az * step;
        }
    }
    qsort(all, n_leaves * nn, 3 * sizeof(int64_t), cmp_key);
    int64_t m = 0;
    for (int64_t i = 0; i < n_leaves * nn; ++i)
        if (m == 0 || cmp_key(all + 3 * (m - 1), all + 3 * i) != 0) {
            memmove(all + 3 * m, all + 3 * i, 3 * sizeof(int64_t));
            ++m;
        }
    O->nnodes = m;
    O->key = realloc(all, sizeof(int64_t) * 3 * m);
    O->cnode = malloc(sizeof(int64_t) * n_leaves * nn);
    for (int64_t e = 0; e < n_leaves; ++e) {
        int64_t step = (int64_t)1 << (max_level - leaves[4 * e]);
        for (int a = 0; a < nn; ++a) {
            int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
            int64_t k[3] = {leaves[4 * e + 1] * O->p + ax * step, leaves[4 * e + 2] * O->p + ay * step,
                            leaves[4 * e + 3] * O->p + az * step};
            O->cnode[e * nn + a] = find_node(O, k);
        }
    }
    /* hanging nodes: on the closed box of a leaf without being one of its nodes */
    int64_t *hang = malloc(sizeof(int64_t) * m);
    for (int64_t k = 0; k < m; ++k) {
        hang[k] = -1;
        const int64_t *x = O->key + 3 * k;
        for (int64_t e = 0; e < n_leaves && hang[k] < 0; ++e) {
            int64_t span = leaf_span(O, e), step = span / O->p;
            int inside = 1, onnode = 1;
            for (int d = 0; d < 3; ++d) {
                int64_t lo = leaves[4 * e + 1 + d] * O->p;
                if (x[d] < lo || x[d] > lo + span) inside = 0;
                else if ((x[d] - lo) % step != 0) onnode = 0;
            }
            if (inside && !onnode) hang[k] = e;
        }
    }
    /* degrees of freedom: regular nodes in key order */
    O->dof = malloc(sizeof(int64_t) * m);
    O->ndofs = 0;
    for (int64_t k = 0; k < m; ++k) O->dof[k] = hang[k] < 0 ? O->ndofs++ : -1;
    O->dnode = malloc(sizeof(int64_t) * (O->ndofs > 0 ? O->ndofs : 1));
    for (int64_t k = 0; k < m; ++k)
        if (O->dof[k] >= 0) O->dnode[O->dof[k]] = k;
    /* closure of every node */
    int64_t **ld = calloc(m, sizeof(int64_t *));
    double **lw = calloc(m, sizeof(double *));
    int64_t *ln = malloc(sizeof(int64_t) * m);
    for (int64_t k = 0; k < m; ++k) ln[k] = -1;
    for (int64_t k = 0; k < m; ++k) expand(O, hang, k, ld, lw, ln);
    O->cs = malloc(sizeof(int64_t) * (m + 1));
    O->cs[0] = 0;
    for (int64_t k = 0; k < m; ++k) O->cs[k + 1] = O->cs[k] + ln[k];
    O->cd = malloc(sizeof(int64_t) * O->cs[m]);
    O->cw = malloc(sizeof(double) * O->cs[m]);
    for (int64_t k = 0; k < m; ++k) {
        memcpy(O->cd + O->cs[k], ld[k], sizeof(int64_t) * ln[k]);
        memcpy(O->cw + O->cs[k], lw[k], sizeof(double) * ln[k]);
        free(ld[k]);
        free(lw[k]);
    }
    free(ld); free(lw); free(ln); free(hang);
    /* lumped mass */
    O->mass = calloc(O->ndofs > 0 ? O->ndofs : 1, sizeof(double));
    for (int64_t e = 0; e < n_leaves; ++e) {
        double x0[3], h[3];
        leaf_geometry(O, e, x0, h);
        double detJ = h[0] * h[1] * h[2];
        for (int a = 0; a < nn; ++a) {
            double me = 0.0;
            for (int q = 0; q < O->R.nq; ++q) me += O->R.wq[q] * detJ * O->R.N[a][q];
            int64_t k = O->cnode[e * nn + a];
            for (int64_t j = O->cs[k]; j < O->cs[k + 1]; ++j) O->mass[O->cd[j]] += O->cw[j] * me;
        }
    }
    return O;
}

int64_t or_oct_n_dofs(const or_octree *O) { return O->ndofs; }
int64_t or_oct_n_hanging(const or_octree *O) { return O->nnodes - O->ndofs; }
int64_t or_oct_n_qp(const or_octree *O) { return O->nl * O->R.nq; }

void or_oct_dof_coords(const or_octree *O, double *xyz)
{
    for (int64_t i = 0; i < O->ndofs; ++i)
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = O->key[3 * O->dnode[i] + d] * O->unit[d] / O->p;
}

static int oct_is_dirichlet(const or_octree *O, int64_t i)
{
    const int64_t *x = O->key + 3 * O->dnode[i];
    int64_t n[3] = {(int64_t)O->P.nx << O->maxl, (int64_t)O->P.ny << O->maxl, O->top};
    unsigned msk = O->P.dirichlet_mask;
    for (int d = 0; d < 3; ++d) {
        if ((msk & (1u << (2 * d))) && x[d] == 0) return 1;
        if ((msk & (2u << (2 * d))) && x[d] == n[d] * O->p) return 1;
    }
    return 0;
}

void or_oct_dirichlet(const or_octree *O, int *flag)
{
    for (int64_t i = 0; i < O->ndofs; ++i) flag[i] = oct_is_dirichlet(O, i);
}

/* initial consolidated fraction per leaf and quadrature point (leaf-major) */
void or_oct_init_history(const or_octree *O, double *rc)
{
    for (int64_t e = 0; e < O->nl; ++e) {
        double x0[3], h[3];
        leaf_geometry(O, e, x0, h);
        for (int q = 0; q < O->R.nq; ++q) {
            double z = x0[2] + O->R.xi[q][2] * h[2];
            rc[e * O->R.nq + q] = (O->P.Lz - z <= O->P.powder_depth) ? 0.0 : 1.0;
        }
    }
}

/* local values of leaf e: the constraint closure applied to the dof vector */
static void gather(const or_octree *O, int64_t e, const double *T, double *Te)
{
    for (int a = 0; a < O->R.nn; ++a) {
        int64_t k = O->cnode[e * O->R.nn + a];
        double v = 0.0;
        for (int64_t j = O->cs[k]; j < O->cs[k + 1]; ++j) v += O->cw[j] * T[O->cd[j]];
        Te[a] = v;
    }
}

static void scatter(const or_octree *O, int64_t e, const double *fe, double *f)
{
    for (int a = 0; a < O->R.nn; ++a) {
        int64_t k = O->cnode[e * O->R.nn + a];
        for (int64_t j = O->cs[k]; j < O->cs[k + 1]; ++j) f[O->cd[j]] += O->cw[j] * fe[a];
    }
}

enum { HIST_UPDATE = 0, HIST_PEEK = 1, HIST_LAGGED = 2 };

/* radiation and evaporation on the face of leaf e at z = Lz, if it has one:
 * fe[a] -= int N_a q_RE(T) dA (eq. bc_rad_evap) */
static void surface_loss_face(const or_octree *O, int64_t e, const double *Te, double *fe)
{
    const ref_elem *R = &O->R;
    const or_problem *P = &O->P;
    int64_t top = O->top;
    if (!or_surface_loss_on(P) || O->leaf[4 * e + 3] + ((int64_t)1 << (O->maxl - O->leaf[4 * e])) != top) return;
    double x0[3], h[3];
    leaf_geometry(O, e, x0, h);
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

/* f_RE(T) alone on the octree (constraint transpose included) */
static void oct_surface_loss_vector(const or_octree *O, const double *T, double *f)
{
    memset(f, 0, sizeof(double) * O->ndofs);
    double Te[MAXNN], fe[MAXNN];
    for (int64_t e = 0; e < O->nl; ++e) {
        gather(O, e, T, Te);
        for (int a = 0; a < O->R.nn; ++a) fe[a] = 0.0;
        surface_loss_face(O, e, Te, fe);
        scatter(O, e, fe, f);
    }
}

/* element vector of leaf e (diffusion + volume source + top-face flux) */
static void oct_cell(const or_octree *O, int64_t e, const double *T, double *rc_cell, int hist, double t,
                     double *fe, double *fv)
{
    /* the implicit residual takes the surface losses lagged at T_n (separately) */
    const int with_re = hist != HIST_LAGGED;
    const ref_elem *R = &O->R;
    const or_problem *P = &O->P;
    double x0[3], h[3];
    leaf_geometry(O, e, x0, h);
    double detJ = h[0] * h[1] * h[2];
    double Te[MAXNN];
    gather(O, e, T, Te);
    for (int a = 0; a < R->nn; ++a) fe[a] = fv[a] = 0.0;
    for (int q = 0; q < R->nq; ++q) {
        double Tq = 0.0, gq[3] = {0, 0, 0};
        for (int a = 0; a < R->nn; ++a) {
            Tq += R->N[a][q] * Te[a];
            for (int d = 0; d < 3; ++d) gq[d] += R->dN[a][q][d] / h[d] * Te[a];
        }
        double r = rc_cell[q];
        double g = or_liquid_fraction(P, Tq);
        double rn = (hist == HIST_LAGGED) ? r : (g > r ? g : r);
        if (hist == HIST_UPDATE) rc_cell[q] = rn;
        double k = or_conductivity(P, Tq, rn);
        double src = or_volume_source(P, x0[0] + R->xi[q][0] * h[0], x0[1] + R->xi[q][1] * h[1],
                                      x0[2] + R->xi[q][2] * h[2], t);
        double W = R->wq[q] * detJ;
        for (int a = 0; a < R->nn; ++a) {
            double gg = 0.0;
            for (int d = 0; d < 3; ++d) gg += R->dN[a][q][d] / h[d] * gq[d];
            fe[a] += W * (-k * gg + R->N[a][q] * src);
            fv[a] += W * R->N[a][q] * src;
        }
    }
    int64_t top = O->top;
    if (P->laser_kind == 0 && O->leaf[4 * e + 3] + ((int64_t)1 << (O->maxl - O->leaf[4 * e])) == top) {
        int n1 = R->n1;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double qs = or_surface_source(P, x0[0] + R->xg[i] * h[0], x0[1] + R->xg[j] * h[1], t);
                double W = R->wg[i] * R->wg[j] * h[0] * h[1];
                for (int a = 0; a < R->nn; ++a) {
                    int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
                    double Na = or_lagrange(P->degree, ax, R->xg[i]) * or_lagrange(P->degree, ay, R->xg[j]) *
                                or_lagrange(P->degree, az, 1.0);
                    fe[a] += W * Na * qs;
                    fv[a] += W * Na * qs;
                }
            }
    }
    if (with_re) surface_loss_face(O, e, Te, fe);
}

int or_oct_assemble(const or_octree *O, const double *T, double *rc, double t, double *f, double *C,
                    double *fvol, int hist)
{
    int64_t N = O->ndofs;
    memset(f, 0, sizeof(double) * N);
    if (fvol) memset(fvol, 0, sizeof(double) * N);
    double fe[MAXNN], fv[MAXNN];
    for (int64_t e = 0; e < O->nl; ++e) {
        oct_cell(O, e, T, rc + e * O->R.nq, hist, t, fe, fv);
        scatter(O, e, fe, f);
        if (fvol) scatter(O, e, fv, fvol);
    }
    for (int64_t i = 0; i < N; ++i) C[i] = O->P.rho * or_capacity(&O->P, T[i]) * O->mass[i];
    return 0;
}

int or_oct_explicit_steps(const or_octree *O, double *T, double *rc, double t0, double dt, int n)
{
    int64_t N = O->ndofs;
    double *f = malloc(sizeof(double) * N), *C = malloc(sizeof(double) * N);
    for (int s = 0; s < n; ++s) {
        or_oct_assemble(O, T, rc, t0 + s * dt, f, C, NULL, HIST_UPDATE);
        for (int64_t i = 0; i < N; ++i) T[i] = oct_is_dirichlet(O, i) ? O->P.T_D : T[i] + dt * f[i] / C[i];
    }
    free(f);
    free(C);
    return 0;
}

/* lambda_max of C~^{-1} K at the critical breakpoint (as or_stability_lambda) */
double or_oct_stability_lambda(const or_octree *O, const double *v0, int iters)
{
    const or_problem *P = &O->P;
    int best = 0;
    for (int i = 1; i < P->n_bp; ++i)
        if (P->k_bp[i] / P->cp_bp[i] > P->k_bp[best] / P->cp_bp[best]) best = i;
    double Tb[1] = {0.0}, kb[1] = {P->k_bp[best]}, cb[1] = {P->cp_bp[best]};
    or_octree L = *O;
    L.P.n_bp = 1;
    L.P.T_bp = Tb;
    L.P.k_bp = kb;
    L.P.cp_bp = cb;
    L.P.latent = 0.0;
    L.P.powder_k_factor = 1.0;
    L.P.laser_kind = -1;
    L.P.emissivity = 0.0; /* the criterion involves K_diff only */
    L.P.evap_on = 0;
    int64_t N = O->ndofs, nq = O->nl * O->R.nq;
    double *v = malloc(sizeof(double) * N), *f = malloc(sizeof(double) * N), *C = malloc(sizeof(double) * N),
           *rc = malloc(sizeof(double) * nq);
    for (int64_t q = 0; q < nq; ++q) rc[q] = 1.0;
    for (int64_t i = 0; i < N; ++i) v[i] = oct_is_dirichlet(O, i) ? 0.0 : v0[i];
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        or_oct_assemble(&L, v, rc, 0.0, f, C, NULL, HIST_UPDATE);
        double num = 0.0, den = 0.0, nrm = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            if (oct_is_dirichlet(O, i)) continue;
            num += -f[i] * v[i];
            den += C[i] * v[i] * v[i];
        }
        lam = num / den;
        for (int64_t i = 0; i < N; ++i) {
            v[i] = oct_is_dirichlet(O, i) ? 0.0 : -f[i] / C[i];
            nrm += v[i] * v[i];
        }
        nrm = sqrt(nrm);
        for (int64_t i = 0; i < N; ++i) v[i] /= nrm;
    }
    free(v); free(f); free(C); free(rc);
    return lam;
}

/* Picard matrix A = C(T_n)/dt + K(T^i) (consistent capacity, lagged history):
 * y = A x and the diagonal sum_e sum_a w_ai^2 A^e_aa (on meshes with hanging
 * nodes this drops the products of two local nodes constrained to the same
 * dof; without hanging nodes it is diag(A)).  Dirichlet entries of x are
 * ignored, Dirichlet rows of y are 0 and of the diagonal 1. */
static void oct_picard(const or_octree *O, const double *Tn, const double *Ti, const double *rc, double dt,
                       const double *x, double *y, double *diag, double *cap_x, const double *xc)
{
    const ref_elem *R = &O->R;
    const or_problem *P = &O->P;
    int64_t N = O->ndofs;
    double *xm = NULL, *xcm = NULL;
    if (x) {
        xm = malloc(sizeof(double) * N);
        for (int64_t i = 0; i < N; ++i) xm[i] = oct_is_dirichlet(O, i) ? 0.0 : x[i];
    }
    if (xc) xcm = (double *)xc;
    if (y) memset(y, 0, sizeof(double) * N);
    if (diag) memset(diag, 0, sizeof(double) * N);
    if (cap_x) memset(cap_x, 0, sizeof(double) * N);
    for (int64_t e = 0; e < O->nl; ++e) {
        double x0[3], h[3];
        leaf_geometry(O, e, x0, h);
        double detJ = h[0] * h[1] * h[2];
        double Tne[MAXNN], Tie[MAXNN], xe[MAXNN], xce[MAXNN], ye[MAXNN], de[MAXNN], ce[MAXNN];
        gather(O, e, Tn, Tne);
        gather(O, e, Ti, Tie);
        if (xm) gather(O, e, xm, xe);
        if (xcm) gather(O, e, xcm, xce);
        for (int a = 0; a < R->nn; ++a) ye[a] = de[a] = ce[a] = 0.0;
        for (int q = 0; q < R->nq; ++q) {
            double Tnq = 0.0, Tiq = 0.0, xq = 0.0, xcq = 0.0, gx[3] = {0, 0, 0};
            for (int b = 0; b < R->nn; ++b) {
                Tnq += R->N[b][q] * Tne[b];
                Tiq += R->N[b][q] * Tie[b];
                if (xm) {
                    xq += R->N[b][q] * xe[b];
                    for (int d = 0; d < 3; ++d) gx[d] += R->dN[b][q][d] / h[d] * xe[b];
                }
                if (xcm) xcq += R->N[b][q] * xce[b];
            }
            double k = or_conductivity(P, Tiq, rc[e * R->nq + q]);
            double m = P->rho * or_capacity(P, Tnq) / dt;
            double W = R->wq[q] * detJ;
            for (int a = 0; a < R->nn; ++a) {
                double gg = 0.0, dd = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double da = R->dN[a][q][d] / h[d];
                    gg += da * gx[d];
                    dd += da * da;
                }
                ye[a] += W * (m * R->N[a][q] * xq + k * gg);
                de[a] += W * (m * R->N[a][q] * R->N[a][q] + k * dd);
                ce[a] += W * m * dt * R->N[a][q] * xcq;
            }
        }
        for (int a = 0; a < R->nn; ++a) {
            int64_t kk = O->cnode[e * R->nn + a];
            for (int64_t j = O->cs[kk]; j < O->cs[kk + 1]; ++j) {
                if (y) y[O->cd[j]] += O->cw[j] * ye[a];
                if (diag) diag[O->cd[j]] += O->cw[j] * O->cw[j] * de[a];
                if (cap_x) cap_x[O->cd[j]] += O->cw[j] * ce[a];
            }
        }
    }
    for (int64_t i = 0; i < N; ++i)
        if (oct_is_dirichlet(O, i)) {
            if (y) y[i] = 0.0;
            if (diag) diag[i] = 1.0;
        }
    free(xm);
}

/* backward-Euler step as or_implicit_step, on the octree */
int or_oct_implicit_step(const or_octree *O, const double *Tn, double *rc, double t, double dt, double cg_rtol,
                         int cg_max_it, double picard_tol, int picard_max_it, double *T_out,
                         int *cg_iters_total, int *picard_iters, double *final_rel_res)
{
    int64_t N = O->ndofs;
    double *Ti = T_out;
    double *res = calloc(N, sizeof(double)), *f = calloc(N, sizeof(double)), *Cl = calloc(N, sizeof(double)),
           *fv = calloc(N, sizeof(double)), *Cx = calloc(N, sizeof(double)), *diag = calloc(N, sizeof(double)),
           *x = calloc(N, sizeof(double)), *r = calloc(N, sizeof(double)), *z = calloc(N, sizeof(double)),
           *p = calloc(N, sizeof(double)), *Ap = calloc(N, sizeof(double)), *dTn = calloc(N, sizeof(double)),
           *fre = calloc(N, sizeof(double));
    oct_surface_loss_vector(O, Tn, fre); /* f_RE lagged at T_n */
    for (int64_t i = 0; i < N; ++i) Ti[i] = oct_is_dirichlet(O, i) ? O->P.T_D : Tn[i];
    int total = 0, status = 0, it;
    double last_rel = 0.0;
    for (it = 0; it < picard_max_it; ++it) {
        or_oct_assemble(O, Ti, rc, t + dt, f, Cl, fv, HIST_LAGGED);
        for (int64_t i = 0; i < N; ++i) dTn[i] = Ti[i] - Tn[i];
        oct_picard(O, Tn, Ti, rc, dt, NULL, NULL, NULL, Cx, dTn);
        double bn = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            res[i] = oct_is_dirichlet(O, i) ? 0.0 : -(Cx[i] / dt - f[i] - fre[i]);
            bn += res[i] * res[i];
        }
        bn = sqrt(bn);
        oct_picard(O, Tn, Ti, rc, dt, NULL, NULL, diag, NULL, NULL);
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
            oct_picard(O, Tn, Ti, rc, dt, p, Ap, NULL, NULL, NULL);
            double pAp = 0.0;
            for (int64_t i = 0; i < N; ++i) pAp += p[i] * Ap[i];
            double alpha = rz / pAp, rz_new = 0.0;
            rr = 0.0;
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
        if (bn > 0 && sqrt(rr) > cg_rtol * bn) status = 1;
        double dmax = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            if (oct_is_dirichlet(O, i)) continue;
            Ti[i] += x[i];
            if (fabs(x[i]) > dmax) dmax = fabs(x[i]);
        }
        if (dmax <= picard_tol) { ++it; break; }
    }
    if (it >= picard_max_it && status == 0) status = 2;
    or_oct_assemble(O, Ti, rc, t + dt, f, Cl, NULL, HIST_UPDATE);
    if (cg_iters_total) *cg_iters_total = total;
    if (picard_iters) *picard_iters = it;
    if (final_rel_res) *final_rel_res = last_rel;
    free(fre);
    free(res); free(f); free(Cl); free(fv); free(Cx); free(diag); free(x); free(r); free(z); free(p); free(Ap);
    free(dTn);
    return status;
}

/* leaf containing a point (the first in leaf order whose closed box holds it)
 * and its reference coordinates */
static int64_t oct_locate(const or_octree *O, const double *pt, double *xi)
{
    for (int64_t e = 0; e < O->nl; ++e) {
        double x0[3], h[3];
        leaf_geometry(O, e, x0, h);
        int in = 1;
        for (int d = 0; d < 3; ++d) {
            double s = (pt[d] - x0[d]) / h[d];
            if (s < -1e-12 || s > 1.0 + 1e-12) in = 0;
            xi[d] = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
        }
        if (in) return e;
    }
    return -1;
}

static double oct_eval(const or_octree *O, int64_t e, const double *xi, const double *T)
{
    double Te[MAXNN], v = 0.0;
    int n1 = O->p + 1;
    gather(O, e, T, Te);
    for (int a = 0; a < O->R.nn; ++a) {
        int ax = a % n1, ay = (a / n1) % n1, az = a / (n1 * n1);
        v += or_lagrange(O->p, ax, xi[0]) * or_lagrange(O->p, ay, xi[1]) * or_lagrange(O->p, az, xi[2]) * Te[a];
    }
    return v;
}

int or_oct_probe(const or_octree *O, const double *T, int n, const double *pts, double *vals)
{
    for (int s = 0; s < n; ++s) {
        double xi[3];
        int64_t e = oct_locate(O, pts + 3 * s, xi);
        if (e < 0) return -1;
        vals[s] = oct_eval(O, e, xi, T);
    }
    return 0;
}

/* Transfer across the adaptation of a growing build (Section 4.1: refinement,
 * coarsening and activation of a new layer).  New dofs inside the old active
 * part take the old finite element field there, dofs above the old top the
 * initial temperature T0 (parts deposited later start at the initial
 * temperature).  A new quadrature point above the old top starts as powder
 * (0 within the powder depth of the new top, 1 below); inside the old part it
 * takes the value of the nearest quadrature point of the old leaf that contains
 * it when the new leaf is that leaf or one of its descendants, and the minimum
 * over all quadrature points of the old leaves inside it when the new leaf is
 * a coarsened parent (unfused powder in any child stays visible). */
int or_oct_transfer_growing(const or_octree *Oo, const double *To, const double *rco, const or_octree *On,
                            double T0, double *Tn, double *rcn)
{
    const double ztop_old = Oo->P.Lz;
    double *xyz = malloc(sizeof(double) * 3 * On->ndofs);
    or_oct_dof_coords(On, xyz);
    for (int64_t i = 0; i < On->ndofs; ++i) {
        double xi[3];
        if (xyz[3 * i + 2] > ztop_old + 1e-12 * ztop_old) { Tn[i] = T0; continue; }
        int64_t e = oct_locate(Oo, xyz + 3 * i, xi);
        if (e < 0) { free(xyz); return -1; }
        Tn[i] = oct_eval(Oo, e, xi, To);
    }
    free(xyz);
    for (int64_t e = 0; e < On->nl; ++e) {
        double x0[3], h[3];
        leaf_geometry(On, e, x0, h);
        const int ln = (int)On->leaf[4 * e];
        for (int q = 0; q < On->R.nq; ++q) {
            double pt[3], xi[3], oxo[3], oh[3];
            for (int d = 0; d < 3; ++d) pt[d] = x0[d] + On->R.xi[q][d] * h[d];
            double *out = rcn + e * On->R.nq + q;
            if (pt[2] > ztop_old) { *out = (On->P.Lz - pt[2] <= On->P.powder_depth) ? 0.0 : 1.0; continue; }
            int64_t eo = oct_locate(Oo, pt, xi);
            if (eo < 0) return -1;
            if (Oo->leaf[4 * eo] > ln) { /* coarsened: minimum over the old leaves inside the new one */
                double m = 1e300;
                for (int64_t f = 0; f < Oo->nl; ++f) {
                    double fx[3], fh[3];
                    leaf_geometry(Oo, f, fx, fh);
                    int in = 1;
                    for (int d = 0; d < 3; ++d)
                        if (fx[d] < x0[d] - 1e-12 * h[d] || fx[d] + fh[d] > x0[d] + h[d] + 1e-12 * h[d]) in = 0;
                    if (!in) continue;
                    for (int qo = 0; qo < Oo->R.nq; ++qo)
                        if (rco[f * Oo->R.nq + qo] < m) m = rco[f * Oo->R.nq + qo];
                }
                *out = m;
                continue;
            }
            leaf_geometry(Oo, eo, oxo, oh);
            int best = 0;
            double bd = 1e300;
            for (int qo = 0; qo < Oo->R.nq; ++qo) {
                double d2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double dx = oxo[d] + Oo->R.xi[qo][d] * oh[d] - pt[d];
                    d2 += dx * dx;
                }
                if (d2 < bd) { bd = d2; best = qo; }
            }
            *out = rco[eo * Oo->R.nq + best];
        }
    }
    return 0;
}

/* Transfer to a new mesh: T_new at each new dof is the old finite element field
 * there.  Each new quadrature point takes the consolidated fraction of the old
 * quadrature point nearest to it in the old leaf that contains it, if that old
 * point lies within the powder depth (so that it tracked the powder state);
 * otherwise the initial value at the new point (0 within the powder depth, 1
 * below): a coarse leaf whose points all lie below the powder layer carries no
 * information about it. */
int or_oct_transfer(const or_octree *Oo, const double *To, const double *rco, const or_octree *On, double *Tn,
                    double *rcn)
{
    double *xyz = malloc(sizeof(double) * 3 * On->ndofs);
    or_oct_dof_coords(On, xyz);
    for (int64_t i = 0; i < On->ndofs; ++i) {
        double xi[3];
        int64_t e = oct_locate(Oo, xyz + 3 * i, xi);
        if (e < 0) { free(xyz); return -1; }
        Tn[i] = oct_eval(Oo, e, xi, To);
    }
    free(xyz);
    for (int64_t e = 0; e < On->nl; ++e) {
        double x0[3], h[3];
        leaf_geometry(On, e, x0, h);
        for (int q = 0; q < On->R.nq; ++q) {
            double pt[3], xi[3], oxo[3], oh[3];
            for (int d = 0; d < 3; ++d) pt[d] = x0[d] + On->R.xi[q][d] * h[d];
            int64_t eo = oct_locate(Oo, pt, xi);
            if (eo < 0) return -1;
            leaf_geometry(Oo, eo, oxo, oh);
            int best = 0;
            double bd = 1e300;
            for (int qo = 0; qo < Oo->R.nq; ++qo) {
                double d2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double dx = oxo[d] + Oo->R.xi[qo][d] * oh[d] - pt[d];
                    d2 += dx * dx;
                }
                if (d2 < bd) { bd = d2; best = qo; }
            }
            const double zo = oxo[2] + Oo->R.xi[best][2] * oh[2];
            if (Oo->P.Lz - zo <= Oo->P.powder_depth) rcn[e * On->R.nq + q] = rco[eo * Oo->R.nq + best];
            else rcn[e * On->R.nq + q] = (On->P.Lz - pt[2] <= On->P.powder_depth) ? 0.0 : 1.0;
        }
    }
    return 0;
}
