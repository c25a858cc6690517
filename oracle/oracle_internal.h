/* Internal declarations shared by the oracle's source files (box and octree
 * meshes).  TEST INFRASTRUCTURE ONLY. */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H

#include "oracle.h"

#define MAXN1 4  /* up to cubic elements */
#define MAXNN 64 /* (p+1)^3 */

/* tensor-product Lagrange element of degree p on [0,1]^3 with the (p+1)^3 Gauss rule */
typedef struct {
    int p, n1, nn, nq;
    double xg[MAXN1], wg[MAXN1];
    double N[MAXNN][MAXNN];     /* N[a][q] */
    double dN[MAXNN][MAXNN][3]; /* reference gradient of N_a at xi_q */
    double wq[MAXNN];           /* tensor quadrature weight (reference cell) */
    double xi[MAXNN][3];        /* reference qp coordinates */
} ref_elem;

int or_make_ref(int p, ref_elem *R);

/* Stefan-Boltzmann constant (exact in the 2019 SI), W m^-2 K^-4 */
#define OR_SIGMA_SB 5.670374419e-8

/* surface losses switched on (radiation or evaporation) */
int or_surface_loss_on(const or_problem *P);

#endif
