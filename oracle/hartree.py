"""The Hartree potential of a density by a finite-element Poisson solve (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

v_H(r) = int rho(r') / |r - r'| dr' is part of the Kohn-Sham Hamiltonian (Sec. 2,
the Hamiltonian after Eq. 3) and, through v_FA = -v_H / N_e, of the initial guess
(Eq. 25). It solves -lap v_H = 4 pi rho. On the orbital mesh, with homogeneous
Dirichlet values on the box and the GLL-lumped right-hand side (Sec. 3.2.1),
    K phi = 4 pi W rho,   i.e. in standard form (K~/2) phi~ = 2 pi W^{1/2} rho,
phi~ = W^{1/2} phi. A charged density's potential does not vanish on the box, so
the monopole is split off first: with Q = int rho and c its centroid,
    rho = Q g_s(r - c) + rho',   g_s the normalised Gaussian of width s,
the Gaussian's potential Q erf(|r - c| / (sqrt(2) s)) / |r - c| is added in closed
form and only rho' (no charge, no dipole about c) is solved for with zero
boundary values. s = 0 solves for rho itself.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla
from scipy.special import erf

from . import fe


def gaussian(X: np.ndarray, c: np.ndarray, s: float) -> np.ndarray:
    """g_s(r - c) = (2 pi s^2)^{-3/2} exp(-|r - c|^2 / (2 s^2)), unit charge."""
    r2 = np.sum((X - c) ** 2, axis=1)
    return np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5


def gaussian_potential(X: np.ndarray, c: np.ndarray, s: float) -> np.ndarray:
    """Potential of g_s: erf(r / (sqrt(2) s)) / r, with its limit sqrt(2/pi)/s at r = 0."""
    r = np.sqrt(np.sum((X - c) ** 2, axis=1))
    out = np.empty_like(r)
    small = r < 1e-8 * s
    out[~small] = erf(r[~small] / (np.sqrt(2.0) * s)) / r[~small]
    out[small] = np.sqrt(2.0 / np.pi) / s
    return out


def hartree(mesh: fe.Mesh3D, rho: np.ndarray, s: float = 0.0):
    """(v_H at the free nodes, Q, c). Direct sparse solve of the Dirichlet problem."""
    X = mesh.coords()
    W = mesh.weights()
    Q = float(W @ rho)
    c = (W * rho) @ X / Q if Q != 0 else np.zeros(3)
    rhs_rho = rho.copy()
    vG = np.zeros_like(rho)
    if s > 0:
        rhs_rho = rho - Q * gaussian(X, c, s)
        vG = Q * gaussian_potential(X, c, s)
    A = fe.kinetic_csr(mesh).tocsc()                  # K~ / 2
    phit = spla.spsolve(A, 2 * np.pi * np.sqrt(W) * rhs_rho)
    return phit / np.sqrt(W) + vG, Q, c
