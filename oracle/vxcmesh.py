"""The exchange-correlation potential on its own linear finite-element mesh (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. 14 puts v_xc on first-order elements, v_xc(r) = sum_b v_b N_b^(1)(r), on a
mesh of its own: uniform of size h_v in an inner cuboid, coarsening towards the
boundary (Sec. 4, finite-element basis). Here that mesh is a tensor product of
three 1-D vertex lists t^x, t^y, t^z covering the orbital box, with trilinear
hat functions N_b^(1) and vertex index b = ix + (m_x + 1)(iy + (m_y + 1) iz).

With the orbital mesh's GLL quadrature (Sec. 3.2.1) the potential enters H only
through its values at the orbital nodes, so the orbital problem sees
    v_a = sum_b N_b^(1)(x_a) u_b,    i.e. v = P u,
and the gradient of Eq. 22 with respect to the linear-mesh unknowns,
    f_b = sum_{k,i} int p psi N_b^(1) = sum_a W_a p_a psi_a N_b^(1)(x_a) = (P^T g)_b,
where g_a = sum_i psi~_{a,i} p~_{a,i} is the nodal gradient of the orbital mesh.

P is assembled here point by point from the hat functions' definition (each
orbital node, the linear cell that contains it, the eight vertex weights).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe, ks


def hat_weights(t: np.ndarray, x: float) -> list[tuple[int, float]]:
    """Nonzero 1-D hat functions at x: [(vertex, N(x))], with t[c] <= x <= t[c+1]."""
    if x < t[0] - 1e-12 or x > t[-1] + 1e-12:
        raise ValueError("point outside the linear mesh")
    c = 0
    while c < t.size - 2 and x > t[c + 1]:
        c += 1
    s = (x - t[c]) / (t[c + 1] - t[c])
    return [(c, 1.0 - s), (c + 1, s)]


def prolongation(mesh: fe.Mesh3D, tx: np.ndarray, ty: np.ndarray, tz: np.ndarray) -> sp.csr_matrix:
    """P (N_f x n_vertices): P[a, b] = N_b^(1)(x_a) (Eq. 14 at the orbital nodes)."""
    X = mesh.coords()
    nx, ny = tx.size, ty.size
    rows, cols, vals = [], [], []
    for a in range(X.shape[0]):
        for ix, wx in hat_weights(tx, X[a, 0]):
            for iy, wy in hat_weights(ty, X[a, 1]):
                for iz, wz in hat_weights(tz, X[a, 2]):
                    rows.append(a)
                    cols.append(ix + nx * (iy + ny * iz))
                    vals.append(wx * wy * wz)
    return sp.csr_matrix((vals, (rows, cols)), shape=(X.shape[0], nx * ny * tz.size))


def evaluate(mesh: fe.Mesh3D, v_fixed: np.ndarray, P: sp.csr_matrix, u: np.ndarray, rho_data: np.ndarray,
             n_elec: int, **kw):
    """L and dL/du for u on the linear mesh: v = v_fixed + P u, f = P^T g (Eqs. 14, 22)."""
    ev = ks.evaluate(mesh, v_fixed + P @ u, rho_data, n_elec, **kw)
    return ev.loss, (P.T @ ev.grad if ev.grad is not None else None), ev
