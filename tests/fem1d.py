"""1D finite element matrices assembled from the closed-form element matrices in
tests/golden/element_matrices_1d.json, and their Kronecker products.

On a uniform axis-aligned box with constant coefficients the 3D stiffness and
mass matrices of the tensor-product Lagrange element are exact Kronecker
products of the 1D ones (Gauss rules with p+1 points integrate these
polynomial integrands exactly).  This gives an assembled-matrix reference that
is independent of the oracle's element loop.
"""
import json
import os

import numpy as np

_G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "element_matrices_1d.json")))


def element_1d(deg, h):
    if deg == 1:
        Me = h / 6.0 * np.array(_G["q1"]["mass_times_6_over_h"], dtype=float)
        Ke = 1.0 / h * np.array(_G["q1"]["stiffness_times_h"], dtype=float)
    elif deg == 2:
        Me = h / 30.0 * np.array(_G["q2"]["mass_times_30_over_h"], dtype=float)
        Ke = 1.0 / (3.0 * h) * np.array(_G["q2"]["stiffness_times_3h"], dtype=float)
    else:
        raise ValueError(deg)
    return Me, Ke


def global_1d(deg, n, h):
    Me, Ke = element_1d(deg, h)
    N = deg * n + 1
    M = np.zeros((N, N))
    K = np.zeros((N, N))
    for c in range(n):
        s = slice(deg * c, deg * c + deg + 1)
        M[s, s] += Me
        K[s, s] += Ke
    return M, K


def global_3d(deg, nx, ny, nz, L):
    """Stiffness K (unit conductivity) and consistent mass M (unit rho*c) on the
    box, nodes numbered x fastest (C order over (z, y, x))."""
    Mx, Kx = global_1d(deg, nx, L[0] / nx)
    My, Ky = global_1d(deg, ny, L[1] / ny)
    Mz, Kz = global_1d(deg, nz, L[2] / nz)
    K = (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) +
         np.kron(Kz, np.kron(My, Mx)))
    M = np.kron(Mz, np.kron(My, Mx))
    return K, M
