"""Closed forms of the decaying eigenmode T = T_D + A sin(pi x) sin(pi y) sin(pi z)
on the unit cube with every face Dirichlet and constant coefficients, computed
from the exact 1D element matrices (tests/golden/element_matrices_1d.json), not
from the oracle or the library.

Q1, uniform h: the nodal sine is an eigenvector of C~^{-1}K (row-sum lumped
mass) with eigenvalue alpha 3 a b^2, a = 2(1 - cos(pi h))/h^2,
b = (2 + cos(pi h))/3, so forward Euler (eq. forward_euler) multiplies it by
(1 - dt alpha lambda) per step.

Q2: the sine sampled at the vertices and at the edge midpoints spans a 2D
subspace that the 1D operators C~^{-1}K and C~^{-1}M leave invariant; in 3D the
evolution is a power of an 8x8 matrix on the Kronecker basis."""
import math

import numpy as np

from tests.fem1d import global_1d


def sine_field(deg, n):
    x = np.linspace(0.0, 1.0, deg * n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)).ravel()


def q1_explicit(n, alpha, dt, nsteps):
    """Nodal field of sin(pi x) sin(pi y) sin(pi z) after nsteps forward-Euler steps (Q1)."""
    h = 1.0 / n
    a = 2.0 / h ** 2 * (1.0 - math.cos(math.pi * h))
    b = (2.0 + math.cos(math.pi * h)) / 3.0
    lam = 3.0 * a * b * b
    return sine_field(1, n) * (1.0 - dt * alpha * lam) ** nsteps


def q2_explicit(n, alpha, dt, nsteps):
    """Nodal field of the same mode after nsteps forward-Euler steps (Q2)."""
    h = 1.0 / n
    M1, K1 = global_1d(2, n, h)
    Ml = M1.sum(axis=1)
    x = np.linspace(0, 1, 2 * n + 1)
    s1 = np.sin(np.pi * x)
    v = s1.copy()
    v[1::2] = 0.0
    m = s1.copy()
    m[0::2] = 0.0
    B = np.stack([v, m], 1)
    inner = slice(1, -1)
    coef = []
    for Op in (K1 / Ml[:, None], M1 / Ml[:, None]):
        Y = Op @ B
        c, *_ = np.linalg.lstsq(B[inner], Y[inner], rcond=None)
        assert np.abs(B[inner] @ c - Y[inner]).max() < 1e-9 * np.abs(Y).max()
        coef.append(c)
    Ak, Am = coef  # Op B = B A on interior rows
    L3 = np.kron(Am, np.kron(Am, Ak)) + np.kron(Am, np.kron(Ak, Am)) + np.kron(Ak, np.kron(Am, Am))
    step = np.eye(8) - dt * alpha * L3
    cN = np.linalg.matrix_power(step, nsteps) @ np.ones(8)  # sine = v + m per direction
    basis = np.kron(B, np.kron(B, B))
    return basis @ cN
