"""Chebyshev filter and Rayleigh-Ritz projection by their plain definitions (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 3.2.2: the spectrum of H~ is mapped by an affine map so that the unwanted
part [a, b] lands on [-1, 1]; the filtered block is Y = p(H~) X with the degree-m
Chebyshev polynomial. We use the normalised filter of Zhou and Saad (2007),
p(lambda) = T_m((lambda - c)/e) / T_m((a0 - c)/e), c = (a+b)/2, e = (b-a)/2,
which is a scalar multiple of T_m of the mapped operator and so spans the same
subspace while keeping the columns O(1).

Rayleigh-Ritz (Eqs. 23-24): the Ritz pairs of H~ in span(Y) are the solutions
of the projected pencil (Y^T H~ Y) u = eps (Y^T Y) u; Ritz vectors Y u.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cheb_T(m: int, x):
    """T_m(x): cos(m arccos x) on [-1, 1], cosh(m arccosh |x|) sign^m outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.cosh(m * np.arccosh(np.abs(xo))) * np.where(xo < 0, (-1.0) ** m, 1.0)
    return out


def filter_scalar(m: int, a: float, b: float, a0: float, lam):
    """The scalar filter p(lambda) = T_m((lambda-c)/e) / T_m((a0-c)/e)."""
    c = 0.5 * (a + b)
    e = 0.5 * (b - a)
    return cheb_T(m, (np.asarray(lam) - c) / e) / cheb_T(m, np.array([(a0 - c) / e]))[0]


def filter_apply(apply_h, X: np.ndarray, m: int, a: float, b: float, a0: float) -> np.ndarray:
    """Y = p(H~) X via the plain three-term Chebyshev recurrence, then normalised.

    T_0 = X, T_1 = (H~ - c) X / e, T_{k+1} = 2 (H~ - c) T_k / e - T_{k-1}; the
    result is T_m / T_m((a0 - c)/e). Plain (unscaled) recurrence, FP64; adequate
    for the degrees used in tests.
    """
    c = 0.5 * (a + b)
    e = 0.5 * (b - a)
    Tkm1 = np.array(X, dtype=np.float64)
    if m == 0:
        return Tkm1.copy()
    Tk = (apply_h(Tkm1) - c * Tkm1) / e
    for _ in range(1, m):
        Tkp1 = 2.0 * (apply_h(Tk) - c * Tk) / e - Tkm1
        Tkm1, Tk = Tk, Tkp1
    return Tk / cheb_T(m, np.array([(a0 - c) / e]))[0]


def rayleigh_ritz(apply_h, Y: np.ndarray):
    """Ritz values and vectors of H~ on span(Y) (Eqs. 23-24), with residual norms."""
    HY = apply_h(Y)
    A = Y.T @ HY
    S = Y.T @ Y
    A = 0.5 * (A + A.T)
    S = 0.5 * (S + S.T)
    w, U = sla.eigh(A, S)
    Psi = Y @ U
    R = HY @ U - Psi * w[None, :]
    return w, Psi, np.linalg.norm(R, axis=0)
